"""Pins for the oracle's advection-diffusion-reaction operator and solve (Remark ADR, Eq. ADR).

Independent anchors:
* physical space: -div(a grad u) + b . grad u + c u evaluated pointwise on a grid (product rule,
  trigonometric sums) and projected by an exact FFT equals the truncated operator applied to a
  u supported on the set (d = 2), for every term at once;
* constant coefficients: the operator is diagonal, u_k = f_k / (4 pi^2 |k|^2 a_0 + 2 pi i k.b_0 + c_0);
* b = 0: the diffusion matrix plus the convolution by c, each built independently;
* the advection part M_b of a real field satisfies M_b + M_b^H = -(div b) as a convolution,
  entry by entry on the set (integration by parts);
* a manufactured solution is recovered by the per-class solve.
"""
import numpy as np
import pytest

from oracle import adr
from oracle import galerkin as og
from oracle import stamp as ost
from tests import _phys


def _real_modes(rng, d, n, lo, hi, width=None, amp=1.0):
    """n random +-w pairs (real trigonometric sums): freqs [2n, d], coefs [2n] or [2n, width]."""
    seen, fr = set(), []
    while len(fr) < n:
        w = rng.integers(lo, hi + 1, size=d)
        t = tuple(int(v) for v in w)
        if not any(t) or t in seen or tuple(-v for v in t) in seen:
            continue
        seen.add(t)
        fr.append(w)
    fr = np.array(fr, dtype=np.int64)
    shape = (n,) if width is None else (n, width)
    c = amp * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    return np.concatenate([fr, -fr]), np.concatenate([c, np.conj(c)])


def _problem(seed, d=2, lo=-3, hi=3):
    rng = np.random.default_rng(seed)
    af, ah = _real_modes(rng, d, 2, lo, hi, amp=0.1)
    af = np.concatenate([np.zeros((1, d), dtype=np.int64), af])
    ah = np.concatenate([[1.5], ah])
    bf, bh = _real_modes(rng, d, 2, lo, hi, width=d, amp=0.2)
    cf, ch = _real_modes(rng, d, 1, lo, hi, amp=0.1)
    cf = np.concatenate([np.zeros((1, d), dtype=np.int64), cf])
    ch = np.concatenate([[2.0], ch])
    F, _ = _real_modes(rng, d, 2, -6, 6)
    return af, ah, bf, bh, cf, ch, F


@pytest.mark.parametrize("seed", range(3))
def test_operator_equals_physical_space_fft_2d(seed):
    af, ah, bf, bh, cf, ch, F = _problem(seed)
    W = adr.support(af, bf, cf, 2)
    keys, _ = ost.stamp(F, W, 2)
    rng = np.random.default_rng(50 + seed)
    u = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    G = 64                      # > twice the largest coordinate of S^2 + supp: no aliasing
    assert np.abs(keys).max() + np.abs(W).max() < G // 2
    pts = _phys.grid_2d(G)
    g = _phys.eval_adr(pts, af, ah, bf, bh, cf, ch, keys, u).reshape(G, G)
    g_hat = _phys.fft_coefficients_2d(g, keys, G)
    Lu = adr.matrix(keys, af, ah, bf, bh, cf, ch) @ u
    # L u on the set holds exactly the terms with k in the set; the projection does too
    assert np.allclose(Lu, g_hat, rtol=0, atol=1e-9 * np.abs(g_hat).max())


def test_constant_coefficients_closed_form():
    d = 3
    keys = np.array([[1, 2, 3], [-1, -2, -3], [4, 0, -1], [0, 5, 0]], dtype=np.int64)
    a0, b0, c0 = 1.3, np.array([0.5, -0.25, 2.0]), 0.7
    z = np.zeros((1, d), dtype=np.int64)
    M = adr.matrix(keys, z, [a0], z, [b0], z, [c0]).toarray()
    diag = 4 * np.pi ** 2 * a0 * (keys ** 2).sum(1) + 2j * np.pi * (keys @ b0) + c0
    assert np.array_equal(M, np.diag(diag)) or np.allclose(M, np.diag(diag), rtol=1e-15, atol=0)
    f = np.array([1.0, 2j, -0.5, 0.25 + 1j])
    u = adr.solve(keys, z, [a0], z, [b0], z, [c0], f)
    assert np.allclose(u, f / diag, rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed", range(2))
def test_no_advection_is_diffusion_plus_reaction(seed):
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=3)
    W = adr.support(af, bf, cf, 3)
    keys, _ = ost.stamp(F, W, 1)
    M = adr.matrix(keys, af, ah, bf, 0 * bh, cf, ch)
    Md = og.matrix(keys, *ost.canonical_a(af, ah))
    # the reaction term as a plain convolution, written out pair by pair
    cmap = {tuple(int(v) for v in w): c for w, c in zip(cf, ch)}
    Mc = np.zeros((len(keys), len(keys)), dtype=np.complex128)
    for i, k in enumerate(keys):
        for m, l in enumerate(keys):
            Mc[i, m] = cmap.get(tuple(int(v) for v in (k - l)), 0.0)
    assert np.allclose(M.toarray(), Md.toarray() + Mc, rtol=0, atol=1e-12 * abs(Md).max())


@pytest.mark.parametrize("seed", range(2))
def test_advection_part_integration_by_parts(seed):
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=3)
    W = adr.support(af, bf, cf, 3)
    keys, _ = ost.stamp(F, W, 1)
    z = np.zeros((1, 3), dtype=np.int64)
    Mb = adr.matrix(keys, z, [0.0], bf, bh, z, [0.0]).toarray()
    bmap = {tuple(int(v) for v in w): c for w, c in zip(bf, bh)}
    div = np.zeros_like(Mb)
    for i, k in enumerate(keys):
        for m, l in enumerate(keys):
            w = k - l
            bw = bmap.get(tuple(int(v) for v in w))
            if bw is not None:
                div[i, m] = 2j * np.pi * np.dot(w.astype(np.float64), bw)
    assert np.allclose(Mb + Mb.conj().T, -div, rtol=0, atol=1e-12 * np.abs(Mb).max())
    assert np.abs(Mb + Mb.conj().T).max() > 1e-3 * np.abs(Mb).max()      # b is not divergence-free


@pytest.mark.parametrize("seed", range(2))
def test_manufactured_solution_recovered(seed):
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=3)
    W = adr.support(af, bf, cf, 3)
    keys, _ = ost.stamp(F, W, 2)
    rng = np.random.default_rng(90 + seed)
    u_star = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    M = adr.matrix(keys, af, ah, bf, bh, cf, ch)
    u = adr.solve(keys, af, ah, bf, bh, cf, ch, M @ u_star, M=M)
    assert np.linalg.norm(u - u_star) <= 1e-10 * np.linalg.norm(u_star)


@pytest.mark.parametrize("seed", range(2))
def test_sparse_class_solve_equals_dense(seed):
    # classes above the dense limit are solved by a sparse LU of the same block: forced on every
    # class here (dense_limit 0), the result equals the dense LU's and a manufactured solution
    af, ah, bf, bh, cf, ch, F = _problem(seed, d=3)
    W = adr.support(af, bf, cf, 3)
    keys, _ = ost.stamp(F, W, 2)
    rng = np.random.default_rng(190 + seed)
    u_star = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    M = adr.matrix(keys, af, ah, bf, bh, cf, ch)
    f = M @ u_star
    u_dense = adr.solve(keys, af, ah, bf, bh, cf, ch, f, M=M)
    u_sparse = adr.solve(keys, af, ah, bf, bh, cf, ch, f, M=M, dense_limit=0)
    assert np.linalg.norm(u_sparse - u_dense) <= 1e-12 * np.linalg.norm(u_dense)
    assert np.linalg.norm(u_sparse - u_star) <= 1e-10 * np.linalg.norm(u_star)
