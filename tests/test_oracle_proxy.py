"""Pins for the oracle's proxy error (Sec. 10.1, Lemma ProxyError): the
relative l2 norm of f - L u^N, with L untruncated, which Prop. LExpansion
places on S^{N+1}.

Independent anchors:
* physical space: f - (-div(a grad u)) evaluated pointwise by the product
  rule (``tests/_phys.py``) on a uniform grid fine enough that no frequency
  of S^{N+1} aliases; the grid mean of |.|^2 is then exactly the sum of the
  squared Fourier coefficients (discrete Parseval), for any u, not only a
  solution (d = 1 and d = 2);
* constant a: the exact solution u_k = f_k / (4 pi^2 a_0 |k|^2) has proxy
  error 0 (textbook Poisson);
* the low-sparsity problem of Sec. 10.3.1 solved on S^N: the proxy error
  falls geometrically in N (Fig. 4a), and the truncated solution of a
  Galerkin solve leaves no residual on S^N itself, so the whole error sits on
  the new level N + 1.
"""
import numpy as np
import pytest

from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests import _phys


def lemma_stamp_decay_rate(af, ah):
    """A / (1 - 2A) of Lemma StampDecay for a coefficient with one cosine mode (|a - a_0|_inf = the
    sum of |a_w| over w != 0, attained; a_min = a_0 minus it); requires 3 |a - a_0|_inf < a_min."""
    zero = ~np.any(np.asarray(af) != 0, axis=1)
    a0 = float(np.real(np.asarray(ah)[zero][0]))
    dev = float(np.abs(np.asarray(ah)[~zero]).sum())
    amin = a0 - dev
    assert 3 * dev < amin
    A = dev / amin
    return A / (1 - 2 * A)


def _setup(p):
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, lev = ost.stamp(p.f_freqs, af, p.level)
    return af, ah, np.asarray(keys), np.asarray(lev)


def _f_on(keys, p):
    pos = og.slot_index(keys)
    f = np.zeros(len(keys), dtype=np.complex128)
    for k, v in zip(p.f_freqs, p.f_hat):
        f[pos[tuple(int(x) for x in k)]] = v
    return f


def _grid_proxy(points, p, af, ah, keys, u):
    r = _phys.eval_series(points, p.f_freqs, p.f_hat) - _phys.eval_operator(points, af, ah, keys, u)
    f = _phys.eval_series(points, p.f_freqs, p.f_hat)
    return np.sqrt(np.mean(np.abs(r) ** 2) / np.mean(np.abs(f) ** 2))


@pytest.mark.parametrize("seed", range(3))
def test_proxy_equals_physical_space_parseval_1d(seed):
    p = workloads.lowsparsity(1, 2 + seed, seed)
    af, ah, keys, _ = _setup(p)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))   # any u, not a solution
    G = 8192                                  # |k| <= 500 + 5 * 500 < 4096: no aliasing
    pts = (np.arange(G) / G)[:, None]
    ref = _grid_proxy(pts, p, af, ah, keys, u)
    got = og.proxy_error(keys, u, af, ah, p.f_freqs, p.f_hat)
    assert abs(got - ref) <= 1e-10 * ref


@pytest.mark.parametrize("level", [1, 2])
def test_proxy_equals_physical_space_parseval_2d(level):
    p = workloads.cfg1(0)                     # a: 4 modes in [-4,4]^2, f in [-8,8]^2
    p.level = level
    af, ah, keys, _ = _setup(p)
    rng = np.random.default_rng(10 + level)
    u = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    G = 64                                    # |k_t| <= 8 + 3 * 4 = 20 < 32: no aliasing
    ref = _grid_proxy(_phys.grid_2d(G), p, af, ah, keys, u)
    got = og.proxy_error(keys, u, af, ah, p.f_freqs, p.f_hat)
    assert abs(got - ref) <= 1e-10 * ref


def test_constant_coefficient_exact_solution_has_zero_proxy():
    d, a0 = 3, 2.5
    af = np.zeros((1, d), dtype=np.int64)
    ah = np.array([a0], dtype=np.complex128)
    F = np.array([[1, -2, 3], [-1, 2, -3], [4, 0, 1], [-4, 0, -1]])
    fh = np.array([0.3 - 0.2j, 0.3 + 0.2j, -1.0j, 1.0j])
    u = fh / (4 * np.pi ** 2 * a0 * (F ** 2).sum(1))
    assert og.proxy_error(F, u, af, ah, F, fh) <= 1e-15
    # a wrong amplitude is seen
    assert og.proxy_error(F, 1.01 * u, af, ah, F, fh) == pytest.approx(0.01, rel=1e-12)


@pytest.mark.parametrize("d", [1, 4, 16])
def test_lowsparsity_proxy_decays_geometrically_and_lives_on_the_new_level(d):
    errs = []
    for N in range(1, 6):
        p = workloads.lowsparsity(d, N)
        af, ah, keys, lev = _setup(p)
        f = _f_on(keys, p)
        u = og.solve(keys, af, ah, f)
        e = og.proxy_error(keys, u, af, ah, p.f_freqs, p.f_hat)
        # the Galerkin residual on S^N vanishes, so |f - L u| is |(L u)| on level N + 1 alone
        nxt, nlev = ost.stamp(p.f_freqs, af, N + 1)
        nxt = np.asarray(nxt)
        top = nxt[np.asarray(nlev) == N + 1]
        pos = og.slot_index(keys)
        Lu_top = []
        for k in top:
            s = 0j
            for w, aw in zip(af, ah):
                l = tuple(int(v) for v in (k - w))
                i = pos.get(l)
                if i is not None:
                    s += 4 * np.pi ** 2 * float(np.dot(k, keys[i])) * aw * u[i]
            Lu_top.append(s)
        assert e == pytest.approx(np.linalg.norm(Lu_top) / np.linalg.norm(p.f_hat), rel=1e-9)
        errs.append(e)
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    # Lemma StampDecay: with A = |a - a_0|_inf / a_min and 3 |a - a_0|_inf < a_min, the truncation
    # error bound shrinks by A / (1 - 2A) per level; for one cosine mode |a - a_0|_inf is the sum of
    # |a_w| over w != 0 and a_min = a_0 minus that sum
    ratio = lemma_stamp_decay_rate(af, ah)
    assert 0 < ratio < 1 and np.all(ratios <= ratio), (ratios, ratio)


def test_highsparsity_workload_and_its_proxy_decay():
    # Sec. 10.3.2: 25 cosine modes with coefficients drawn once and kept for every d, a_0 = 4 ceil(|c|_2)
    # (so the l1 certificate holds), f = sin(2 pi k_f.x); the exact proxy error falls with the level
    c_ref = None
    for d in (1, 4, 64):
        p = workloads.highsparsity(d, 1)
        af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
        assert len(af) == 51 and np.all(np.abs(p.a_freqs) <= 500)
        z = np.all(af == 0, axis=1)
        c = np.sort(2 * ah[~z].real)
        assert np.all(ah[~z].imag == 0)
        c_ref = c if c_ref is None else c_ref
        assert np.array_equal(c, c_ref)                  # the same coefficients for every d
        assert ah[z][0].real == 4 * np.ceil(np.linalg.norm(c) / np.sqrt(2))
        assert p.a_min_bound() > 0
        assert sorted(p.f_hat.tolist(), key=lambda v: v.imag) == [-0.5j, 0.5j]
    errs = []
    for N in range(3):
        p = workloads.highsparsity(4, N)
        af, ah, keys, lev = _setup(p)
        f = _f_on(keys, p)
        u = og.solve(keys, af, ah, f)
        errs.append(og.proxy_error(keys, u, af, ah, p.f_freqs, p.f_hat))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.5 * errs[0]
