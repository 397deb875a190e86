"""Pins for the oracle's solve (Alg. 1, steps 3-5; Sec. 9 Eq.
SparseSpectralSFTEquation).

Independent anchors:
* manufactured solutions: u* chosen on S^N, f = -div(a grad u*) computed in
  physical space and projected by an exact FFT (d = 2), then recovered;
* constant a: u_k = f_k / (4 pi^2 |k|^2 a_0) (Poisson, textbook);
* one cosine mode in d = 1: a tridiagonal system, solved by the Thomas
  algorithm written out here;
* real f gives u_{-k} = conj(u_k); the energy <f,u> is real and positive;
  the stability bound |u|_H <= |f| / a_min (Prop. ExistenceUniquenessStability);
* the level-block identity (Cor. after Prop. LExpansion) for the truncated
  system;
* dense LU and the CG fallback agree.
"""
import numpy as np
import pytest

from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads
from tests import _phys
from tests.test_oracle_operator import _random_problem


def _f_on_slots(keys, f_freqs, f_hat):
    pos = og.slot_index(keys)
    f = np.zeros(len(keys), dtype=np.complex128)
    for k, v in zip(np.asarray(f_freqs), f_hat):
        f[pos[tuple(int(x) for x in k)]] = v
    return f


@pytest.mark.parametrize("seed", range(3))
def test_manufactured_solution_fft_2d(seed):
    rng = np.random.default_rng(100 + seed)
    af, ah, F = _random_problem(rng, 2, 4, 4, -4, 4, amp=0.4)
    keys, _ = ost.stamp(F, af, 2)
    u_star = workloads.manufactured_solution(len(keys), seed, density=0.5)
    u_star[~np.any(keys != 0, axis=1)] = 0
    G = 64
    g = _phys.eval_operator(_phys.grid_2d(G), af, ah, keys, u_star).reshape(G, G)
    f = _phys.fft_coefficients_2d(g, keys, G)       # (L u*) restricted to S^N
    zero = ~np.any(keys != 0, axis=1)
    assert np.all(np.abs(f[zero]) <= 1e-12 * np.abs(f).max())   # a divergence has mean 0
    f[zero] = 0
    u = og.solve(keys, af, ah, f)
    assert np.linalg.norm(u - u_star) <= 1e-11 * np.linalg.norm(u_star)


def test_constant_coefficient_closed_form():
    rng = np.random.default_rng(4)
    F = rng.integers(-20, 21, size=(9, 4))
    F = F[np.any(F != 0, axis=1)]
    keys, _ = ost.stamp(F, np.zeros((1, 4), dtype=np.int64), 0)
    f = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    u = og.solve(keys, np.zeros((1, 4), dtype=np.int64), np.array([3.0]), f)
    assert np.allclose(u, f / (4 * np.pi ** 2 * 3.0 * (keys ** 2).sum(1)), rtol=1e-14, atol=0)


def _thomas(lower, diag, upper, rhs):
    """Textbook tridiagonal elimination (no pivoting)."""
    n = len(diag)
    c = np.zeros(n, dtype=np.complex128)
    dd = np.zeros(n, dtype=np.complex128)
    c[0] = upper[0] / diag[0]
    dd[0] = rhs[0] / diag[0]
    for i in range(1, n):
        den = diag[i] - lower[i] * c[i - 1]
        c[i] = upper[i] / den if i < n - 1 else 0
        dd[i] = (rhs[i] - lower[i] * dd[i - 1]) / den
    x = np.zeros(n, dtype=np.complex128)
    x[-1] = dd[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dd[i] - c[i] * x[i + 1]
    return x


def test_one_mode_1d_is_tridiagonal():
    # -(a u')' = f with a = a0 + c cos(2 pi m x) + phase: the Fourier coefficient
    # of (a u')' couples k only to k +- m, so on the chain k_f + j m (|j| <= N)
    # the Galerkin system is tridiagonal with entries 4 pi^2 k l a_{k-l}.
    m, kf, N, a0 = 3, 5, 6, 2.0
    am = 0.4 * np.exp(0.7j)                       # a_{+m}; a_{-m} = conj
    af = np.array([[-m], [0], [m]])
    ah = np.array([np.conj(am), a0, am])
    keys, _ = ost.stamp(np.array([[kf]]), af, N)
    assert keys[:, 0].tolist() == [kf + j * m for j in range(-N, N + 1)]
    rng = np.random.default_rng(0)
    f = rng.standard_normal(len(keys)) + 1j * rng.standard_normal(len(keys))
    k = keys[:, 0].astype(np.float64)
    c = 4 * np.pi ** 2
    diag = c * k * k * a0
    lower = np.concatenate([[0], c * k[1:] * k[:-1] * am])           # a_{k-l}, k-l = +m
    upper = np.concatenate([c * k[:-1] * k[1:] * np.conj(am), [0]])  # k-l = -m
    ref = _thomas(lower, diag, upper, f)
    u = og.solve(keys, af, ah, f)
    assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("config", [1, 3])
def test_real_forcing_symmetry_energy_stability(config):
    p = workloads.make(config)
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, af, min(p.level, 2))
    f = _f_on_slots(keys, p.f_freqs, p.f_hat)
    u = og.solve(keys, af, ah, f)
    pos = og.slot_index(keys)
    neg = np.array([pos[tuple(-int(v) for v in k)] for k in keys])   # S is symmetric here
    assert np.max(np.abs(u[neg] - np.conj(u))) <= 1e-13 * np.abs(u).max()
    e = np.vdot(u, f)                                # <f, u> = <L u, u>
    assert e.real > 0 and abs(e.imag) <= 1e-12 * e.real
    a_min = 0.125 if config == 3 else _phys.eval_series(_phys.grid_2d(256), af, ah).real.min()
    h_norm = np.sqrt((4 * np.pi ** 2 * (keys ** 2).sum(1) * np.abs(u) ** 2).sum())
    assert h_norm <= np.linalg.norm(f) / a_min


def test_level_block_identity():
    # b_{m,n} = <L_N u|_m, u|_n>; for n < N, b_{n+1,n} + b_{n,n} + b_{n-1,n} equals
    # <f, u|_{level n}>; at the top level the (absent) n+1 term drops out.
    p = workloads.make(2, level=2)
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, lev = ost.stamp(p.f_freqs, af, p.level)
    f = _f_on_slots(keys, p.f_freqs, p.f_hat)
    M = og.matrix(keys, af, ah)
    u = og.solve(keys, af, ah, f, M=M)
    part = [np.where(lev == n, u, 0) for n in range(p.level + 1)]
    b = lambda m, n: np.vdot(part[n], M @ part[m]) if 0 <= m <= p.level else 0.0
    for n in range(p.level + 1):
        lhs = b(n + 1, n) + b(n, n) + b(n - 1, n)
        rhs = np.vdot(part[n], f)
        assert abs(lhs - rhs) <= 1e-12 * abs(np.vdot(u, f))
    # and the off-level terms vanish (Prop. LExpansion)
    assert abs(b(2, 0)) == 0.0 and abs(b(0, 2)) == 0.0


def test_dense_and_cg_agree():
    p = workloads.make(1)
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, af, p.level)
    f = _f_on_slots(keys, p.f_freqs, p.f_hat)
    u1 = og.solve(keys, af, ah, f)
    u2 = og.solve(keys, af, ah, f, dense_limit=0)
    assert np.linalg.norm(u1 - u2) <= 1e-12 * np.linalg.norm(u1)


def test_mean_zero_required():
    keys = np.array([[-1, 0], [0, 0], [1, 0]])
    with pytest.raises(ValueError):
        og.solve(keys, np.zeros((1, 2), dtype=np.int64), np.array([1.0]), np.array([1.0, 1.0, 1.0]))
