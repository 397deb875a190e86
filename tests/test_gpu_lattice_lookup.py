"""GPU: neighbour lookups by rank-1 lattice value (ss_build_op's default: lat(k - w) = lat(k) - lat(w)
mod M, no key read) give the oracle's neighbour map bit for bit and the same operator as the
key-comparing lookups (SS_EXACT_LOOKUP), at d = 2 .. 1024, so the solutions are bitwise equal."""
import numpy as np
import pytest

from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests.test_gpu_parity import FLAGS, _wide_problem, f_vector, gpu_solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_00752_amd import sparsespec
    return sparsespec


CASES = {
    "cfg1": lambda: [workloads.make(1, 0)],
    "cfg2": lambda: [workloads.make(2, i) for i in range(3)],
    "cfg3": lambda: [workloads.make(3, 0)],
    "cfg4": lambda: [workloads.make(4, i) for i in range(2)],
    "wide70": lambda: [_wide_problem(70, 50, seed=70)],
    "high1024": lambda: [workloads.highsparsity(1024, 2, i) for i in range(2)],
    "low1024": lambda: [workloads.lowsparsity(1024, n, 5) for n in (1, 3, 5)],
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_lattice_lookup_equals_oracle_and_key_lookup(ss, case):
    probs = CASES[case]()
    flags = FLAGS.get(3, 0) if case == "cfg3" else 0
    st = ss.Stamp.build(probs)
    op_k = ss.Operator.build(st, probs, flags | ss.SS_EXACT_LOOKUP)
    op_l = ss.Operator.build(st, probs, flags)
    ck, cl = op_k.csr(), op_l.csr()
    for a, b in zip(ck, cl):
        assert np.array_equal(a, b)
    assert np.array_equal(op_k.exec_map(), op_l.exec_map())
    keys, _ = st.keys()
    # the oracle's map for the first problem (the others are checked through the equality above)
    p = probs[0]
    af, _ = ost.canonical_a(p.a_freqs, p.a_hat)
    okeys, _ = ost.stamp(p.f_freqs, af, p.level)
    n0 = len(okeys)
    assert np.array_equal(keys[:n0].astype(np.int64), okeys)
    orp, ocols, ojs = og.neighbours(okeys, af)
    rp, cols, js, _ = cl
    assert np.array_equal(rp[:n0 + 1], orp)
    assert np.array_equal(cols[:orp[-1]], ocols) and np.array_equal(js[:orp[-1]], ojs)
    f = f_vector(ss, st, probs)
    uk, _ = gpu_solve(ss, op_k, f, 1e-11, "fp64")
    ul, _ = gpu_solve(ss, op_l, f, 1e-11, "fp64")
    assert np.array_equal(uk, ul)
