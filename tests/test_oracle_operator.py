"""Pins for the oracle's Galerkin operator (Sec. 5 Eq. GF; Sec. 9 Eq.
FiniteGalerkinOperator) and its neighbour relation.

Independent anchors:
* the PDE operator -div(a grad u) evaluated in physical space by the product
  rule (``tests/_phys.py``), then projected on S^N by an exact FFT (d = 2) or
  compared pointwise on S^{N+1}, where no truncation happens (Prop.
  LExpansion: L maps level n into levels n-1..n+1);
* constant a: the Poisson operator 4 pi^2 |k|^2 a_0 (textbook);
* Hermitian symmetry and the Rayleigh bounds a_min <= <Lx,x>/|x|_H^2 <= a_max
  (Prop. ExistenceUniquenessStability, Prop. GalerkinBilinearForm);
* level locality of the neighbour relation (Prop. LExpansion) and the
  closed-form entry count and class structure in generic position.
"""
import math

import numpy as np
import pytest

from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests import _phys


def _random_problem(rng, d, half, n_f, lo, hi, a0=1.0, amp=0.3):
    modes = []
    seen = set()
    while len(modes) < half:
        w = tuple(int(v) for v in rng.integers(lo, hi + 1, size=d))
        if any(w) and w not in seen and tuple(-v for v in w) not in seen:
            seen.add(w)
            modes.append(w)
    modes = np.array(modes)
    c = rng.standard_normal(half) + 1j * rng.standard_normal(half)
    c *= amp / (2 * np.abs(c).sum())
    af = np.concatenate([np.zeros((1, d), dtype=np.int64), modes, -modes])
    ah = np.concatenate([[a0], c, np.conj(c)])
    F = []
    seenf = set()
    while len(F) < n_f:
        k = tuple(int(v) for v in rng.integers(lo, hi + 1, size=d))
        if any(k) and k not in seenf:
            seenf.add(k)
            F.append(k)
    return ost.canonical_a(af, ah) + (np.array(F),)


@pytest.mark.parametrize("seed", range(3))
def test_matvec_equals_fft_projection_2d(seed):
    rng = np.random.default_rng(seed)
    af, ah, F = _random_problem(rng, 2, 4, 5, -4, 4)
    keys, _ = ost.stamp(F, af, 2)
    x = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    y = og.apply(keys, af, ah, x)
    G = 64                                    # |freq| <= 4 + 2*4 + 4 < 32: no aliasing
    g = _phys.eval_operator(_phys.grid_2d(G), af, ah, keys, x).reshape(G, G)
    ref = _phys.fft_coefficients_2d(g, keys, G)
    assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,half,n_f,N", [(10, 3, 3, 2), (100, 4, 2, 1), (3, 5, 2, 2)])
def test_matvec_pointwise_on_next_level(d, half, n_f, N):
    rng = np.random.default_rng(d)
    af, ah, F = _random_problem(rng, d, half, n_f, -8, 8)
    keys, _ = ost.stamp(F, af, N)
    big, _ = ost.stamp(F, af, N + 1)
    x = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    pos = og.slot_index(big)
    xb = np.zeros(len(big), dtype=np.complex128)
    idx = np.array([pos[tuple(int(v) for v in k)] for k in keys])
    xb[idx] = x
    yb = og.apply(big, af, ah, xb)            # = L x exactly: supp(Lx) within S^{N+1}
    pts = rng.random((40, d))
    lhs = _phys.eval_series(pts, big, yb)
    rhs = _phys.eval_operator(pts, af, ah, keys, x)
    assert np.max(np.abs(lhs - rhs)) <= 1e-10 * np.max(np.abs(rhs))
    # truncation: L_N x is the restriction of L x to S^N (l outside S^N carry x_l = 0)
    assert np.allclose(og.apply(keys, af, ah, x), yb[idx], rtol=0, atol=1e-12 * np.abs(yb).max())


def test_constant_coefficient_is_poisson():
    rng = np.random.default_rng(2)
    d = 5
    F = rng.integers(-9, 10, size=(7, d))
    af = np.zeros((1, d), dtype=np.int64)
    keys, _ = ost.stamp(F, af, 3)
    x = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    y = og.apply(keys, af, np.array([2.5]), x)
    assert np.allclose(y, 4 * np.pi ** 2 * 2.5 * (keys ** 2).sum(1) * x, rtol=1e-15, atol=0)


@pytest.mark.parametrize("config", [1, 2, 3])
def test_hermitian_and_rayleigh_bounds(config):
    p = workloads.make(config)
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, af, min(p.level, 2))
    M = og.matrix(keys, af, ah)
    assert abs(M - M.getH()).max() == 0.0                   # exactly Hermitian
    rng = np.random.default_rng(config)
    nz = np.any(keys != 0, axis=1)
    if config == 3:                                         # closed form of the product
        a_lo, a_hi = 0.5 ** 3, 1.5 ** 3
    elif config == 1:                                       # sampled on a fine grid
        vals = _phys.eval_series(_phys.grid_2d(256), af, ah).real
        a_lo, a_hi = vals.min(), vals.max()
    else:                                                   # l1 certificate
        a0 = ah[np.all(af == 0, axis=1)][0].real
        dev = np.abs(ah).sum() - a0
        a_lo, a_hi = a0 - dev, a0 + dev
    for _ in range(5):
        x = (rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))) * nz
        e = np.vdot(x, M @ x)
        hn = (4 * np.pi ** 2 * (keys ** 2).sum(1) * np.abs(x) ** 2).sum()
        assert abs(e.imag) <= 1e-12 * abs(e.real)
        assert a_lo * (1 - 1e-12) <= e.real / hn <= a_hi * (1 + 1e-12)


def test_level_locality_and_symmetric_relation():
    for config in (1, 2, 3):
        p = workloads.make(config)
        af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
        keys, lev = ost.stamp(p.f_freqs, af, min(p.level, 2))
        rp, cols, js = og.neighbours(keys, af)
        rows = np.repeat(np.arange(len(keys)), np.diff(rp))
        assert np.all(np.abs(lev[rows] - lev[cols]) <= 1)
        assert set(zip(rows.tolist(), cols.tolist())) == set(zip(cols.tolist(), rows.tolist()))
        # js follows the a-table and gives k - l = w_j
        assert np.array_equal(keys[rows] - keys[cols], af[js])


@pytest.mark.parametrize("d,half,n_f,N", [(40, 5, 6, 3), (12, 4, 3, 2)])
def test_entry_count_and_classes_in_generic_position(d, half, n_f, N):
    rng = np.random.default_rng(d + N)
    A = rng.integers(-10 ** 4, 10 ** 4, size=(half, d))
    af = np.concatenate([np.zeros((1, d), dtype=np.int64), A, -A])
    F = rng.integers(-10 ** 4, 10 ** 4, size=(n_f, d))
    keys, lev = ost.stamp(F, af, N)
    rp, cols, _ = og.neighbours(keys, af)
    s = 2 * half + 1
    # rows below level N see all s neighbours; a level-N row built from t
    # distinct +-w directions sees itself and one step back along each
    top = n_f * sum(2 ** t * math.comb(half, t) * math.comb(N - 1, t - 1) * (1 + t)
                    for t in range(1, min(N, half) + 1))
    assert len(cols) == ost.cardinality_bound(n_f, s, N - 1) * s + top
    label = og.classes(rp, cols)
    sizes = np.unique(label, return_counts=True)[1]
    assert len(sizes) == n_f and np.all(sizes == len(keys) // n_f)
