"""GPU parity of the rank-1 lattice entry point (Sec. 8, Definition of a reconstructing rank-1
lattice, Lemma RandomRank1Lattice) through the C ABI against the oracle.

Bars: lattice indices k . z mod M bit-exact; the per-problem reconstructing flag equal to the
oracle's Definition check -- at the Lemma's modulus, at moduli too small to separate the set
(pigeonhole) and at moduli where some draws of z fail; the batch of the timed workload
(512 d = 10 problems, 16 M keys) with sampled problems checked one by one; the argument errors.
"""
import numpy as np
import pytest

from oracle import lattice as ol
from paper_2302_00752_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_00752_amd import sparsespec
    return sparsespec


def _sets(st):
    keys, _ = st.keys()
    return [keys[st.offsets[i]:st.offsets[i + 1]].astype(np.int64) for i in range(st.n_prob)]


CASES = {
    "cfg1": lambda: [workloads.cfg1(0), workloads.cfg1(1)],
    "cfg2": lambda: [workloads.cfg2(0)],
    "cfg3": lambda: [workloads.cfg3(0, level=2)],
    "d1024": lambda: [workloads.lowsparsity(1024, 2, 0), workloads.lowsparsity(1024, 3, 1)],
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_values_and_flags_match_oracle(ss, case):
    probs = CASES[case]()
    st = ss.Stamp.build(probs)
    sets = _sets(st)
    n = max(len(s) for s in sets)
    K = max(ol.expansion(s) for s in sets)
    rng = np.random.default_rng(31)
    # the Lemma's modulus, one at the birthday scale (some draws fail), one below the set size
    for M in (ss.lattice_modulus(K, n, 0.01), ol.next_prime(max(K, n * n // 8)), ol.next_prime(max(2, n // 2))):
        for _ in range(3):
            z = rng.integers(1, M, size=st.d)
            ok, vals = st.lattice(z, M)
            torch.cuda.synchronize()
            v = vals.cpu().numpy()
            for i, s in enumerate(sets):
                assert np.array_equal(v[st.offsets[i]:st.offsets[i + 1]], ol.lattice_values(s, z, M)), (case, M, i)
                assert bool(ok[i]) == ol.is_reconstructing(s, z, M), (case, M, i)
                if M < len(s):
                    assert not ok[i]


def test_flags_without_values_and_edge_moduli(ss):
    st = ss.Stamp.build([workloads.cfg1(0)])
    s = _sets(st)[0]
    z = np.ones(st.d, dtype=np.int64)
    ok, vals = st.lattice(z, 2, values=False)
    assert vals is None and not ok[0]            # two lattice points, hundreds of frequencies
    M = 1 << 40                                  # the largest modulus accepted
    z = np.random.default_rng(32).integers(1, M, size=st.d)
    ok, vals = st.lattice(z, M)
    torch.cuda.synchronize()
    assert np.array_equal(vals.cpu().numpy(), ol.lattice_values(s, z, M))
    assert bool(ok[0]) == ol.is_reconstructing(s, z, M)


def test_argument_errors(ss):
    st = ss.Stamp.build([workloads.cfg1(0)])
    for z, M in (([0, 1], 11), ([1, 11], 11), ([1, 2], 1), ([1, 2], (1 << 40) + 1)):
        with pytest.raises(ss.SparseSpecError) as e:
            st.lattice(np.array(z), M)
        assert e.value.status == ss.SS_EINVAL, (z, M)
    with pytest.raises(ss.SparseSpecError):
        st.lattice(np.array([1, 2, 3]), 11)


def test_full_batch_sampled_against_oracle(ss):
    # the timed workload's stamp: 512 d = 10 problems of 31 220 keys; the Lemma's modulus at
    # sigma = 0.01 for one set, one z for the batch
    probs = [workloads.make(2, i) for i in range(512)]
    st = ss.Stamp.build(probs)
    keys, _ = st.keys()
    n = 31220
    assert np.all(np.diff(st.offsets) == n)
    K = int((keys.max(axis=0).astype(np.int64) - keys.min(axis=0)).max())
    M = ss.lattice_modulus(K, n, 0.01)
    z = np.random.default_rng(33).integers(1, M, size=10)
    ok, vals = st.lattice(z, M)
    torch.cuda.synchronize()
    v = vals.cpu().numpy()
    # each set fails with probability below sigma: at most a few of 512
    assert (~ok).sum() <= 20
    sample = sorted({0, 255, 511} | set(np.flatnonzero(~ok)[:3].tolist()))
    for i in sample:
        s = keys[st.offsets[i]:st.offsets[i + 1]].astype(np.int64)
        assert np.array_equal(v[st.offsets[i]:st.offsets[i + 1]], ol.lattice_values(s, z, M)), i
        assert bool(ok[i]) == ol.is_reconstructing(s, z, M), i
