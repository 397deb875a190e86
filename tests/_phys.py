"""Physical-space evaluation of the PDE operator, independent of the oracle.

For trigonometric polynomials a(x) = sum_w a_w e_w(x) and u(x) = sum_k u_k e_k(x),
e_k(x) = exp(2 pi i k.x) (Sec. 3), the strong form of the operator (Sec. 4,
Def. EllipticPDE) is expanded with the product rule,
    -div(a grad u) = -grad a . grad u - a lap u,
and every factor is evaluated pointwise from its trigonometric sum.  Nothing
here forms a Galerkin coefficient.
"""
import numpy as np


def eval_operator(points, a_freqs, a_hat, u_freqs, u_hat):
    pts = np.asarray(points, dtype=np.float64)
    wf = np.asarray(a_freqs, dtype=np.float64)
    kf = np.asarray(u_freqs, dtype=np.float64)
    Ea = np.exp(2j * np.pi * pts @ wf.T)                   # [P, s]
    Eu = np.exp(2j * np.pi * pts @ kf.T)                   # [P, n]
    a = Ea @ a_hat
    grad_a = Ea @ (2j * np.pi * wf * a_hat[:, None])       # [P, d]
    grad_u = Eu @ (2j * np.pi * kf * u_hat[:, None])       # [P, d]
    lap_u = Eu @ (-4 * np.pi ** 2 * (kf ** 2).sum(1) * u_hat)
    return -(grad_a * grad_u).sum(1) - a * lap_u


def eval_series(points, freqs, coef):
    pts = np.asarray(points, dtype=np.float64)
    return np.exp(2j * np.pi * pts @ np.asarray(freqs, dtype=np.float64).T) @ coef


def fft_coefficients_2d(g_on_grid, keys, G):
    """Fourier coefficients of a grid function at integer frequencies ``keys``."""
    gh = np.fft.fft2(g_on_grid) / (G * G)
    keys = np.asarray(keys)
    return gh[keys[:, 0] % G, keys[:, 1] % G]


def grid_2d(G):
    x = np.arange(G) / G
    X, Y = np.meshgrid(x, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def eval_adr(points, a_freqs, a_hat, b_freqs, b_hat, c_freqs, c_hat, u_freqs, u_hat):
    """-div(a grad u) + b . grad u + c u pointwise (Remark ADR, Eq. ADR); b_hat[i] is the
    vector of the d components' coefficients at b_freqs[i]."""
    pts = np.asarray(points, dtype=np.float64)
    kf = np.asarray(u_freqs, dtype=np.float64)
    Eu = np.exp(2j * np.pi * pts @ kf.T)
    grad_u = Eu @ (2j * np.pi * kf * u_hat[:, None])                    # [P, d]
    u = Eu @ u_hat
    bf = np.asarray(b_freqs, dtype=np.float64)
    b = np.exp(2j * np.pi * pts @ bf.T) @ np.asarray(b_hat)            # [P, d]
    c = eval_series(pts, c_freqs, np.asarray(c_hat))
    return eval_operator(pts, a_freqs, a_hat, u_freqs, u_hat) + (b * grad_u).sum(1) + c * u
