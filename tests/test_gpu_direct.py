"""GPU parity of the dense direct solve (Alg. 1, steps 4-5, per connected class of Sec. 6):
tiled Cholesky in FP64 through the C ABI against the oracle's per-class dense solve.

Bars: |u - u_oracle| / |u_oracle| <= 1e-10 at the paper's configurations (cfg2 at its full
level 3: 20 classes of 1561 rows, 49 tiles each), the residual |f - L u| / |f| <= 1e-12 by
the FP64 matvec, agreement with FP64 PCG, each problem bitwise the same in a batch as alone,
u_0 = 0, classes too large for the substitution's LDS vector, and the error paths (a class above
the row limit, an indefinite operator).  The FP32
factorisation with FP64 refinement to a residual of 1e-12 meets the same bars.
"""
import numpy as np
import pytest

from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests.test_gpu_parity import (ERR64, FLAGS, P, build, f_vector, oracle_case, rel)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_00752_amd import sparsespec
    return sparsespec


def direct(ss, op, f, precision="fp64", tol=0.0):
    fd = torch.from_numpy(f).cuda()
    ud = torch.full_like(fd, complex(np.nan, np.nan))
    info = op.solve_direct(fd, ud, precision, tol)
    torch.cuda.synchronize()
    return ud.cpu().numpy(), info


def residual(ss, op, f, u):
    em = op.exec_map()
    ue = np.zeros(op.n_exec, dtype=np.complex128)
    ue[em >= 0] = u[em[em >= 0]]
    xd = torch.from_numpy(ue).cuda()
    yd = torch.zeros_like(xd)
    op.apply(xd, yd, "fp64")
    torch.cuda.synchronize()
    y = np.zeros(op.n_total, dtype=np.complex128)
    y[em[em >= 0]] = yd.cpu().numpy()[em >= 0]
    return np.linalg.norm(f - y) / np.linalg.norm(f)


@pytest.mark.parametrize("case", [(1, None), (2, 2), (2, None), (4, 1)])
def test_direct_matches_oracle(ss, case):
    config, level = case
    oc = oracle_case(config, 0, level)
    st, op = build(ss, [oc["p"]], FLAGS.get(config, 0))
    f = f_vector(ss, st, [oc["p"]])
    u, info = direct(ss, op, f)
    sizes = op.class_sizes()
    assert sizes.sum() == op.n_total and len(sizes) == op.n_components
    assert np.array_equal(np.sort(sizes), np.sort(np.unique(oc["label"], return_counts=True)[1]))
    nt = (sizes + 31) // 32
    assert info["tiles"] == int((nt * (nt + 1) // 2).sum()) and info["chunks"] >= 1
    assert rel(u, oc["u"]) <= ERR64, rel(u, oc["u"])
    assert residual(ss, op, f, u) <= 1e-12
    assert np.all(u[~np.any(oc["keys"] != 0, axis=1)] == 0)


def test_direct_full_level_classes_and_pcg(ss):
    # d = 10 at level 3 (the matvec workload's problem): 20 classes of 1561 rows; the direct
    # solution agrees with FP64 PCG run to 1e-13
    oc = oracle_case(2)
    st, op = build(ss, [oc["p"]])
    sizes = op.class_sizes()
    assert sizes.max() == 1561 and len(sizes) == 20
    f = f_vector(ss, st, [oc["p"]])
    u, _ = direct(ss, op, f)
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    op.solve(fd, ud, 1e-13, "fp64", 5000)
    torch.cuda.synchronize()
    assert rel(u, ud.cpu().numpy()) <= 1e-11


def test_direct_batch_equals_alone_bitwise(ss):
    # classes are factored independently: a problem's u does not depend on its batch or chunk
    probs = [workloads.make(2, i, level=2) for i in range(3)] + [workloads.make(1, 0), workloads.make(4, 0, level=1)]
    batch = [p for p in probs if p.d == 10]
    st, op = build(ss, batch)
    u, _ = direct(ss, op, f_vector(ss, st, batch))
    for i, p in enumerate(batch):
        s1, o1 = build(ss, [p])
        ua, _ = direct(ss, o1, f_vector(ss, s1, [p]))
        assert np.array_equal(u[st.offsets[i]:st.offsets[i + 1]], ua), i
    for p in probs[3:]:
        s1, o1 = build(ss, [p])
        f = f_vector(ss, s1, [p])
        ua, _ = direct(ss, o1, f)
        af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
        keys, _ = ost.stamp(p.f_freqs, af, p.level)
        assert rel(ua, og.solve(keys, af, ah, f)) <= ERR64


def test_direct_edge_cases(ss):
    # one key; d = 1 tridiagonal; k = 0 inside the set (zero row and column, u_0 = 0); int64 norms
    cases = [P(1, [[0]], [1.5], [[7]], [2.0], 3),
             P(1, [[0], [3], [-3]], [2.0, 0.4 + 0.3j, 0.4 - 0.3j], [[5], [-5]], [1j, -1j], 6),
             P(2, [[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1]], [1.0, 0.2, 0.2, 0.1j, -0.1j],
               [[1, 0], [-1, 0]], [1.0, 1.0], 2),
             P(3, [[0, 0, 0], [1, 2, 0], [-1, -2, 0], [0, 1, 3], [0, -1, -3]],
               [2.0, 0.3 + 0.2j, 0.3 - 0.2j, 0.25j, -0.25j],
               [[30000, -29000, 31000], [-30000, 29000, -31000], [29990, 29995, -30001]],
               [1.0 + 1j, 1.0 - 1j, 0.5], 2)]
    for p in cases:
        af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
        keys, _ = ost.stamp(p.f_freqs, af, p.level)
        st, op = build(ss, [p])
        f = f_vector(ss, st, [p])
        u, _ = direct(ss, op, f)
        assert rel(u, og.solve(keys, af, ah, f)) <= ERR64
        assert np.all(u[~np.any(keys != 0, axis=1)] == 0)


def test_direct_one_class_of_thousands_of_rows(ss):
    # a dense support in d = 2 merges the set into a few classes of several thousand rows
    w = [(1, 0), (0, 1), (1, 1), (2, -1)]
    af = [[0, 0]] + [list(v) for v in w] + [[-a, -b] for a, b in w]
    ah = [1.0] + [0.05 + 0.02j] * 4 + [0.05 - 0.02j] * 4
    p = P(2, af, ah, [[3, 1], [-3, -1], [5, -7], [-5, 7]], [1.0, 1.0, 0.3j, -0.3j], 16)
    st, op = build(ss, [p])
    assert op.class_sizes().max() > 2048
    f = f_vector(ss, st, [p])
    u, _ = direct(ss, op, f)
    a2, h2 = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, a2, p.level)
    assert rel(u, og.solve(keys, a2, h2, f)) <= ERR64
    assert residual(ss, op, f, u) <= 1e-12


def test_direct_errors(ss):
    # a class above the 32 768-row limit: a dense support in d = 2 at level 78, one class of 36 815 rows
    w = [(1, 0), (0, 1), (1, 1), (2, -1)]
    af = [[0, 0]] + [list(v) for v in w] + [[-a, -b] for a, b in w]
    ah = [1.0] + [0.05 + 0.02j] * 4 + [0.05 - 0.02j] * 4
    p = P(2, af, ah, [[3, 1]], [1.0], 78)
    st, op = build(ss, [p])
    assert op.class_sizes().max() == 36815
    f = torch.from_numpy(f_vector(ss, st, [p])).cuda()
    with pytest.raises(ss.SparseSpecError) as e:
        op.solve_direct(f, torch.zeros_like(f))
    assert e.value.status == ss.SS_ERANGE
    # a = 0.1 + cos(2 pi x) changes sign: with the positivity check skipped the block is
    # indefinite and the factorisation reports it
    p = P(1, [[0], [1], [-1]], [0.1, 0.5, 0.5], [[1], [-1]], [1.0, 1.0], 6)
    st, op = build(ss, [p], 1)
    f = torch.from_numpy(f_vector(ss, st, [p])).cuda()
    with pytest.raises(ss.SparseSpecError) as e:
        op.solve_direct(f, torch.zeros_like(f))
    assert e.value.status == ss.SS_ENOTPD


@pytest.mark.parametrize("d", [1, 4, 1024])
def test_direct_high_sparsity(ss, d):
    # the high-sparsity problem of Sec. 10.3.2 at level 2 (two classes of 1301 rows for d > 1, one
    # merged class for d = 1; d = 1024: 2 KB keys, int64 norms): direct = PCG (and = the oracle at
    # small d), residual at rounding level
    p = workloads.highsparsity(d, 2)
    st, op = build(ss, [p])
    f = f_vector(ss, st, [p])
    u, _ = direct(ss, op, f)
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    op.solve(fd, ud, 1e-13, "fp64", 5000)
    torch.cuda.synchronize()
    assert rel(u, ud.cpu().numpy()) <= 1e-11
    assert residual(ss, op, f, u) <= 1e-12
    if d <= 4:
        af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
        keys, _ = ost.stamp(p.f_freqs, af, p.level)
        assert rel(u, og.solve(keys, af, ah, f)) <= ERR64


def test_direct_class_near_the_row_limit(ss):
    # one class of 7919 rows (248 tile rows, 506 MB of tiles, the substitution's class vector
    # filling 144 KB of LDS), below the 8192-row limit: residual at rounding level, PCG agrees
    w = [(1, 0), (0, 1), (1, 1), (2, -1)]
    af = [[0, 0]] + [list(v) for v in w] + [[-a, -b] for a, b in w]
    ah = [1.0] + [0.05 + 0.02j] * 4 + [0.05 - 0.02j] * 4
    p = P(2, af, ah, [[3, 1]], [1.0 + 0.5j], 36)
    st, op = build(ss, [p])
    sizes = op.class_sizes()
    assert sizes.max() == 7919 and len(sizes) == 1
    f = f_vector(ss, st, [p])
    u, info = direct(ss, op, f)
    assert info["tiles"] == 248 * 249 // 2
    assert residual(ss, op, f, u) <= 1e-12
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    op.solve(fd, ud, 1e-13, "fp64", 20000)
    torch.cuda.synchronize()
    assert rel(u, ud.cpu().numpy()) <= 1e-9
    # and against the oracle (its textbook CG above 6000 rows, to 1e-15)
    afo, aho = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, afo, p.level)
    assert len(keys) == 7919
    assert rel(u, og.solve(keys, afo, aho, f)) <= ERR64


@pytest.mark.parametrize("case", [(1, None), (2, 2), (2, None), (4, 1)])
def test_direct_fp32_refine_matches_oracle(ss, case):
    config, level = case
    oc = oracle_case(config, 0, level)
    st, op = build(ss, [oc["p"]], FLAGS.get(config, 0))
    f = f_vector(ss, st, [oc["p"]])
    u, info = direct(ss, op, f, "fp32_refine", 1e-12)
    assert info["refine_steps"] >= 2 and info["rel_residual"] <= 1e-12
    assert rel(u, oc["u"]) <= ERR64, (rel(u, oc["u"]), info)
    assert residual(ss, op, f, u) <= 1e-12
    assert np.all(u[~np.any(oc["keys"] != 0, axis=1)] == 0)
    # FP64 with the same tolerance: one step already meets it
    u64, i64 = direct(ss, op, f, "fp64", 1e-12)
    assert i64["refine_steps"] == 1 and i64["rel_residual"] <= 1e-12


def test_direct_fp32_refine_batch_equals_alone_and_limits(ss):
    # refinement stops per class, so each problem's u is bitwise its solve alone
    probs = [workloads.make(2, i, level=2) for i in range(3)]
    st, op = build(ss, probs)
    u, _ = direct(ss, op, f_vector(ss, st, probs), "fp32_refine", 1e-12)
    for i, p in enumerate(probs):
        s1, o1 = build(ss, [p])
        ua, _ = direct(ss, o1, f_vector(ss, s1, [p]), "fp32_refine", 1e-12)
        assert np.array_equal(u[st.offsets[i]:st.offsets[i + 1]], ua), i
    # a tolerance below rounding is reported, the last iterate kept
    p = workloads.make(1, 0)
    s1, o1 = build(ss, [p])
    f = f_vector(ss, s1, [p])
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    with pytest.raises(ss.SparseSpecError) as e:
        o1.solve_direct(fd, ud, "fp32_refine", 1e-30)
    assert e.value.status == ss.SS_ENOCONV
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, af, p.level)
    assert rel(ud.cpu().numpy(), og.solve(keys, af, ah, f)) <= ERR64


def test_direct_classes_beyond_lds(ss):
    # the high-sparsity problem at level 3: two classes of 22 151 rows (693 tile rows), whose
    # substitution keeps the class vector in device memory; FP32 factor refined in FP64
    p = workloads.highsparsity(4, 3)
    st, op = build(ss, [p])
    sizes = op.class_sizes()
    assert len(sizes) == 2 and sizes.min() == sizes.max() == 22151
    f = f_vector(ss, st, [p])
    u, info = direct(ss, op, f, "fp32_refine", 1e-12)
    assert info["rel_residual"] <= 1e-12 and info["refine_steps"] >= 2
    assert residual(ss, op, f, u) <= 1e-12
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    op.solve(fd, ud, 1e-13, "fp64", 5000)
    torch.cuda.synchronize()
    assert rel(u, ud.cpu().numpy()) <= 1e-9
    # and against the oracle (its textbook CG for classes this size, to 1e-15)
    afo, aho = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, afo, p.level)
    assert rel(u, og.solve(keys, afo, aho, f)) <= ERR64
