"""GPU parity of the advection-diffusion-reaction path (Remark ADR, Eq. ADR) through the C ABI
against the oracle's ADR operator and per-class dense solve.

Bars: stamp keys on the union support bit-exact; the matvec within 64 eps64 |L| |x| per row;
BiCGSTAB solutions within |u - u_oracle| / |u_oracle| <= 1e-10 (tol 1e-12); a manufactured
solution recovered; each problem bitwise the same in a batch as alone; the argument errors.
"""
import numpy as np
import pytest

from oracle import adr
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests.test_gpu_parity import f_vector, rel
from tests.test_oracle_adr import _problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_00752_amd import sparsespec
    return sparsespec


def _from_pins(seed, level):
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=3)
    rng = np.random.default_rng(300 + seed)
    fh = rng.standard_normal(len(F) // 2) + 1j * rng.standard_normal(len(F) // 2)
    fh = np.concatenate([fh, np.conj(fh)])
    return workloads.AdrProblem(3, af.astype(np.int16), ah, bf.astype(np.int16), bh, cf.astype(np.int16), ch,
                                F.astype(np.int16), fh, level)


def build(ss, problems):
    dps = [p.diffusion_on_union() for p in problems]
    st = ss.Stamp.build(dps)
    op = ss.Operator.build(st, dps, 0)
    A = ss.AdrOperator.build(st, op, problems)
    return st, op, A, dps


def oracle_of(p):
    W = adr.support(p.a_freqs, p.b_freqs, p.c_freqs, p.d)
    keys, _ = ost.stamp(p.f_freqs, W, p.level)
    M = adr.matrix(keys, p.a_freqs, p.a_hat, p.b_freqs, p.b_hat, p.c_freqs, p.c_hat)
    return keys, M


def gpu_solve(A, f, tol=1e-12, max_iter=4000):
    fd = torch.from_numpy(f).cuda()
    ud = torch.full_like(fd, complex(np.nan, np.nan))
    info = A.solve(fd, ud, tol, max_iter)
    torch.cuda.synchronize()
    return ud.cpu().numpy(), info


@pytest.mark.parametrize("case", ["adr3d-1", "pins-2"])
def test_adr_stamp_and_apply(ss, case):
    p = workloads.adr3d(1) if case == "adr3d-1" else _from_pins(0, 2)
    keys, M = oracle_of(p)
    st, op, A, _ = build(ss, [p])
    gk, _ = st.keys()
    assert np.array_equal(gk.astype(np.int64), keys)
    em = op.exec_map()
    rng = np.random.default_rng(5)
    x = rng.standard_normal(op.n_total) + 1j * rng.standard_normal(op.n_total)
    xe = np.zeros(op.n_exec, dtype=np.complex128)
    xe[em >= 0] = x[em[em >= 0]]
    xd = torch.from_numpy(xe).cuda()
    yd = torch.full_like(xd, complex(np.nan, np.nan))
    A.apply(xd, yd)
    torch.cuda.synchronize()
    ye = yd.cpu().numpy()
    assert np.all(ye[em < 0] == 0)
    y = np.zeros(op.n_total, dtype=np.complex128)
    y[em[em >= 0]] = ye[em >= 0]
    bound = abs(M) @ np.abs(x)
    assert np.all(np.abs(y - M @ x) <= 64 * np.finfo(np.float64).eps * bound + 1e-300)


@pytest.mark.parametrize("case", ["adr3d-1", "adr3d-2", "pins-1", "pins-2"])
def test_adr_solve_matches_oracle(ss, case):
    # adr3d: the paper's data size (45 operator terms, an 89-entry union support; at level 2 one
    # class of about 4e4 rows, which the oracle solves by a sparse LU)
    kind, lv = case.split("-")
    p = workloads.adr3d(int(lv)) if kind == "adr3d" else _from_pins(1, int(lv))
    if kind == "adr3d":
        assert len(p.union()) == 89
    keys, M = oracle_of(p)
    st, op, A, dps = build(ss, [p])
    f = f_vector(ss, st, dps)
    u, info = gpu_solve(A, f)
    assert info[0]["status"] == ss.SS_OK and info[0]["rel_residual"] <= 1e-12
    u_ref = adr.solve(keys, p.a_freqs, p.a_hat, p.b_freqs, p.b_hat, p.c_freqs, p.c_hat, f, M=M)
    assert rel(u, u_ref) <= 1e-10, (rel(u, u_ref), info)


def test_adr_manufactured_solution(ss):
    p = workloads.adr3d(1, 3)
    keys, M = oracle_of(p)
    st, op, A, _ = build(ss, [p])
    u_star = workloads.manufactured_solution(len(keys), 11, density=0.3)
    u, info = gpu_solve(A, M @ u_star)
    assert rel(u, u_star) <= 1e-10 and info[0]["status"] == ss.SS_OK


def test_adr_batch_equals_alone_bitwise(ss):
    probs = [workloads.adr3d(1, i) for i in range(3)] + [workloads.adr3d(2, 7)]
    st, op, A, dps = build(ss, probs)
    u, info = gpu_solve(A, f_vector(ss, st, dps))
    for i, p in enumerate(probs):
        s1, o1, a1, d1 = build(ss, [p])
        ua, ia = gpu_solve(a1, f_vector(ss, s1, d1))
        assert np.array_equal(u[st.offsets[i]:st.offsets[i + 1]], ua), i
        assert ia[0]["iters"] == info[i]["iters"]


def test_adr_argument_errors(ss):
    p = workloads.adr3d(1)
    dps = [p.diffusion_on_union()]
    st = ss.Stamp.build(dps)
    op = ss.Operator.build(st, dps, 0)
    bad_c = workloads.AdrProblem(**{**p.__dict__, "c_freqs": p.c_freqs[1:], "c_hat": p.c_hat[1:]})
    with pytest.raises(ss.SparseSpecError) as e:
        ss.AdrOperator.build(st, op, [bad_c])
    assert e.value.status == ss.SS_EINVAL
    far = np.array([[49, 49, 49], [-49, -49, -49]], dtype=np.int16)
    assert not any((w == far[0]).all() for w in p.union())
    bad_b = workloads.AdrProblem(**{**p.__dict__, "b_freqs": np.concatenate([p.b_freqs, far]),
                                    "b_hat": np.concatenate([p.b_hat, np.ones((2, 3))])})
    with pytest.raises(ss.SparseSpecError) as e:
        ss.AdrOperator.build(st, op, [bad_b])
    assert e.value.status == ss.SS_EINVAL


def _small(seed, d, lo=-3, hi=3, far=0):
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=d, lo=lo, hi=hi)
    F = F + far * np.sign(F + 0.5).astype(np.int64)     # push F out to coordinates near `far`
    rng = np.random.default_rng(700 + seed)
    fh = rng.standard_normal(len(F) // 2) + 1j * rng.standard_normal(len(F) // 2)
    fh = np.concatenate([fh, np.conj(fh)])
    return workloads.AdrProblem(d, af.astype(np.int16), ah, bf.astype(np.int16), bh, cf.astype(np.int16), ch,
                                F.astype(np.int16), fh, 2)


@pytest.mark.parametrize("d,far", [(1, 0), (16, 0), (3, 30000)])
def test_adr_other_dimensions_and_int64_norms(ss, d, far):
    # d = 1 (one merged class), d = 16, and coordinates near 3e4 in d = 3 (|k|^2 > 2^30: int64 norms)
    p = _small(d, d, far=far)
    if far:
        assert 3 * (far - 10) ** 2 > 2 ** 30
    keys, M = oracle_of(p)
    st, op, A, dps = build(ss, [p])
    f = f_vector(ss, st, dps)
    u, info = gpu_solve(A, f)
    u_ref = adr.solve(keys, p.a_freqs, p.a_hat, p.b_freqs, p.b_hat, p.c_freqs, p.c_hat, f, M=M)
    assert info[0]["status"] == ss.SS_OK and rel(u, u_ref) <= 1e-10, (rel(u, u_ref), info)
