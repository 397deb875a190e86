"""Seeded synthetic PDE data for the sparse spectral Galerkin solver.

This module only draws inputs: sparse Fourier data of a real, strictly
positive diffusion coefficient ``a`` and of a real, mean-zero forcing ``f`` on
the d-torus (Sec. 4, Def. of the elliptic PDE; Sec. 5, Galerkin form).  It
holds none of the method's arithmetic (no stamp sets, no operator, no solve);
both the CPU oracle and the HIP path consume what it returns.

Conventions (Sec. 3): ``e_k(x) = exp(2 pi i k.x)``, so a real term
``c cos(2 pi w.x + phi)`` has coefficients ``c/2 e^{i phi}`` at ``w`` and
``c/2 e^{-i phi}`` at ``-w``, and ``c sin(2 pi w.x)`` has ``-i c/2`` at ``w`` and
``+i c/2`` at ``-w``.

Workload recipes (all seeded with numpy PCG64, ``seed = 1000*config + instance``):

* ``cfg1``  d=2,  a = 1 + sum_{j<4} 0.2 cos(2 pi w_j.x + phi_j), w_j in [-4,4]^2,
  redrawn until a >= 0.5 on a 256^2 grid; f: 5 real modes in [-8,8]^2 with
  N(0,1) complex amplitudes (|F| = 10); stamp level 2.
* ``cfg2``  d=10, a_0 = 1, 10 modes w ~ U([-16,16]^10), |a_w| ~ U(0,1)/|w|^2 with
  random phase, non-constant part scaled to l1 <= 0.5 (so a in [0.5, 1.5]);
  f: 10 real modes in [-16,16]^10 (|F| = 20); level 3.
* ``cfg3``  d=3, a(x) = prod_j (1 + 0.5 sin(2 pi K_j x_j)), K = (1, 32, 512)
  (27 coefficients, a in [0.125, 3.375]); f: 20 real modes in [-64,64]^3
  (|F| = 40); level 3.
* ``cfg4``  d=100, 20 cosine modes, each with 5 nonzero coordinates drawn from
  {-8..8}\\{0}, amplitudes 0.1 N(0,1) scaled to l1 <= 0.5; f: 20 real modes of
  the same law (|F| = 40); level 2.
* ``cfg5``  serving requests: d ~ U{2..50}, 5..20 a- and f-modes with min(d,5)
  nonzero coordinates in {-8..8}\\{0}, level chosen so the stamp set holds
  1e3..1e5 frequencies, precision FP64 or FP32+refine with probability 1/2,
  Poisson arrival times.
* ``lowsparsity``  the exactly sparse low-sparsity problem of Sec. 10.3.1:
  a = 4 + c_a cos(2 pi k_a.x) with c_a ~ U[-1, 1] drawn once per instance and
  kept for every d (as the paper does), f = sin(2 pi k_f.x), k_a and k_f ~
  U([-499, 500]^d), nonzero and k_f != +-k_a; any d (the paper runs d = 1 to
  1024) and level N (the paper: N = 1..5).  Seeds ``7000 + instance`` for c_a and
  ``7000 + 10007 d + instance`` for the frequencies.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Problem:
    """Sparse Fourier data of one periodic elliptic problem.

    ``a_freqs`` [s, d] int16 and ``a_hat`` [s] complex128 list the full support of
    the diffusion coefficient (closed under negation, containing 0);
    ``f_freqs`` [m, d] int16 and ``f_hat`` [m] complex128 the forcing support.
    """
    d: int
    a_freqs: np.ndarray
    a_hat: np.ndarray
    f_freqs: np.ndarray
    f_hat: np.ndarray
    level: int
    name: str = ""
    precision: str = "fp64"     # "fp64" or "fp32_refine" (serving requests)
    arrival_s: float = 0.0      # serving arrival time in seconds

    def a_min_bound(self) -> float:
        """Lower bound a_0 - ||a - a_0||_1 on a (valid when positive)."""
        z = np.all(self.a_freqs == 0, axis=1)
        a0 = float(self.a_hat[z][0].real)
        return a0 - float(np.abs(self.a_hat[~z]).sum())


def _rng(config: int, instance: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


def _distinct_modes(rng, n, draw_one, forbid=()):
    """Draw ``n`` nonzero modes, pairwise distinct and not opposite."""
    seen = set(tuple(int(v) for v in f) for f in forbid)
    out = []
    while len(out) < n:
        w = np.asarray(draw_one(), dtype=np.int64)
        t = tuple(int(v) for v in w)
        nt = tuple(-v for v in t)
        if not any(t) or t in seen or nt in seen:
            continue
        seen.add(t)
        out.append(w)
    return np.stack(out)


def _real_from_half(d, modes, amps, a0=None):
    """Full conjugate-symmetric list from one representative per +-w pair.

    ``amps[j]`` is the coefficient at ``modes[j]``; ``conj(amps[j])`` goes to
    ``-modes[j]``.  ``a0`` (if given) is the real coefficient at 0.
    """
    freqs = [modes, -modes]
    coef = [amps, np.conj(amps)]
    if a0 is not None:
        freqs.insert(0, np.zeros((1, d), dtype=np.int64))
        coef.insert(0, np.array([a0], dtype=np.complex128))
    return (np.concatenate(freqs).astype(np.int16),
            np.concatenate(coef).astype(np.complex128))


def _grid_min_2d(a_freqs, a_hat, n=256):
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    val = np.zeros_like(X)
    for w, c in zip(a_freqs.astype(np.float64), a_hat):
        val += (c * np.exp(2j * np.pi * (w[0] * X + w[1] * Y))).real
    return float(val.min())


def _forcing(rng, d, n_modes, draw_one, forbid=()):
    modes = _distinct_modes(rng, n_modes, draw_one, forbid)
    amps = rng.standard_normal(n_modes) + 1j * rng.standard_normal(n_modes)
    return _real_from_half(d, modes, amps)


def cfg1(instance: int = 0) -> Problem:
    rng = _rng(1, instance)
    d = 2
    while True:
        modes = _distinct_modes(rng, 4, lambda: rng.integers(-4, 5, size=d))
        phi = rng.uniform(0, 2 * np.pi, size=4)
        af, ah = _real_from_half(d, modes, 0.1 * np.exp(1j * phi), a0=1.0)
        if _grid_min_2d(af, ah) >= 0.5:
            break
    ff, fh = _forcing(rng, d, 5, lambda: rng.integers(-8, 9, size=d))
    return Problem(d, af, ah, ff, fh, level=2, name=f"cfg1/{instance}")


def cfg2(instance: int = 0, level: int = 3) -> Problem:
    rng = _rng(2, instance)
    d = 10
    modes = _distinct_modes(rng, 10, lambda: rng.integers(-16, 17, size=d))
    mag = rng.uniform(0, 1, size=10) / (modes.astype(np.float64) ** 2).sum(1)
    amps = mag * np.exp(1j * rng.uniform(0, 2 * np.pi, size=10))
    l1 = 2 * np.abs(amps).sum()
    if l1 > 0.5:
        amps *= 0.5 / l1
    af, ah = _real_from_half(d, modes, amps, a0=1.0)
    ff, fh = _forcing(rng, d, 10, lambda: rng.integers(-16, 17, size=d))
    return Problem(d, af, ah, ff, fh, level=level, name=f"cfg2/{instance}")


def cfg3(instance: int = 0, level: int = 3) -> Problem:
    rng = _rng(3, instance)
    d = 3
    K = (1, 32, 512)
    c = {0: 1.0 + 0j, 1: -0.25j, -1: 0.25j}   # 1 + 0.5 sin(2 pi K x)
    freqs, coefs = [], []
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for l in (-1, 0, 1):
                freqs.append((i * K[0], j * K[1], l * K[2]))
                coefs.append(c[i] * c[j] * c[l])
    af = np.array(freqs, dtype=np.int16)
    ah = np.array(coefs, dtype=np.complex128)
    ff, fh = _forcing(rng, d, 20, lambda: rng.integers(-64, 65, size=d))
    return Problem(d, af, ah, ff, fh, level=level, name=f"cfg3/{instance}")


def _nonzero_sparse_mode(rng, d, nnz):
    w = np.zeros(d, dtype=np.int64)
    idx = rng.choice(d, size=nnz, replace=False)
    mag = rng.integers(1, 9, size=nnz)
    sgn = rng.choice(np.array([-1, 1]), size=nnz)
    w[idx] = mag * sgn
    return w


def cfg4(instance: int = 0, level: int = 2) -> Problem:
    rng = _rng(4, instance)
    d = 100
    modes = _distinct_modes(rng, 20, lambda: _nonzero_sparse_mode(rng, d, 5))
    c = 0.1 * rng.standard_normal(20)
    amps = (c / 2).astype(np.complex128)
    l1 = 2 * np.abs(amps).sum()
    if l1 > 0.5:
        amps *= 0.5 / l1
    af, ah = _real_from_half(d, modes, amps, a0=1.0)
    ff, fh = _forcing(rng, d, 20, lambda: _nonzero_sparse_mode(rng, d, 5))
    return Problem(d, af, ah, ff, fh, level=level, name=f"cfg4/{instance}")


def generic_stamp_size(n_f: int, s: int, level: int) -> int:
    """Stamp-set size when no frequency coincidences occur (App. A count).

    Used only to size serving requests before drawing them; the exact set is
    built by the solver.  ``s`` counts 0, so ``(s-1)/2`` cosine pairs.
    """
    half = (s - 1) // 2
    total = 0
    for n in range(level + 1):
        for t in range(0, min(n, half) + 1):
            if n == 0 and t == 0:
                total += 1
            elif t >= 1:
                total += 2 ** t * math.comb(half, t) * math.comb(n - 1, t - 1)
    return n_f * total


def cfg5_request(rng: np.random.Generator, rid: int,
                 size_lo: int = 1000, size_hi: int = 100000) -> Problem:
    """One serving request (drawn until its generic stamp size is in range)."""
    while True:
        d = int(rng.integers(2, 51))
        na = int(rng.integers(5, 21))
        nf = int(rng.integers(5, 21))
        nz = min(d, 5)
        modes = _distinct_modes(rng, na, lambda: _nonzero_sparse_mode(rng, d, nz))
        c = 0.1 * rng.standard_normal(na)
        amps = (c / 2).astype(np.complex128)
        l1 = 2 * np.abs(amps).sum()
        if l1 > 0.5:
            amps *= 0.5 / l1
        af, ah = _real_from_half(d, modes, amps, a0=1.0)
        ff, fh = _forcing(rng, d, nf, lambda: _nonzero_sparse_mode(rng, d, nz))
        s = af.shape[0]
        level = 0
        for n in (1, 2, 3):
            if generic_stamp_size(ff.shape[0], s, n) <= size_hi:
                level = n
        if level == 0 or generic_stamp_size(ff.shape[0], s, level) < size_lo:
            continue
        prec = "fp64" if rng.random() < 0.5 else "fp32_refine"
        return Problem(d, af, ah, ff, fh, level=level,
                       name=f"cfg5/{rid}", precision=prec)


def cfg5_stream(n_requests: int = 1024, rate_per_s: float = 1000.0,
                instance: int = 0, size_lo: int = 1000,
                size_hi: int = 100000) -> List[Problem]:
    """A serving stream: requests with Poisson arrival times."""
    rng = _rng(5, instance)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        p = cfg5_request(rng, i, size_lo, size_hi)
        p.arrival_s = t
        out.append(p)
    return out


def manufactured_solution(n: int, seed: int, density: float = 0.3,
                          zero_index: Optional[int] = None) -> np.ndarray:
    """A sparse random coefficient vector on ``n`` slots (for manufactured tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u[rng.random(n) > density] = 0
    if zero_index is not None:
        u[zero_index] = 0
    return u


def lowsparsity(d: int, level: int, instance: int = 0) -> Problem:
    c_a = float(np.random.Generator(np.random.PCG64(7000 + instance)).uniform(-1.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(7000 + 10007 * d + instance))
    draw = lambda: rng.integers(-499, 501, size=d)
    k_a = _distinct_modes(rng, 1, draw)
    k_f = _distinct_modes(rng, 1, draw, forbid=k_a)
    af, ah = _real_from_half(d, k_a, np.array([c_a / 2], dtype=np.complex128), a0=4.0)
    ff, fh = _real_from_half(d, k_f, np.array([-0.5j], dtype=np.complex128))
    return Problem(d, af, ah, ff, fh, level=level, name=f"lowsparsity/d{d}/N{level}/{instance}")


def highsparsity(d: int, level: int, instance: int = 0) -> Problem:
    """The exactly sparse high-sparsity diffusion problem (Sec. 10.3.2): a = a_0 + sum over 25 modes
    k of c_k cos(2 pi k.x), c ~ U[-1, 1]^25 drawn once and kept for every d and instance, a_0 =
    4 ceil(|c|_2); f = sin(2 pi k_f.x); every frequency uniform in [-499, 500]^d (instance picks
    the frequencies)."""
    c = np.random.Generator(np.random.PCG64(8000)).uniform(-1.0, 1.0, size=25)
    rng = np.random.Generator(np.random.PCG64(8000 + 10007 * d + instance))
    draw = lambda: rng.integers(-499, 501, size=d)
    k_a = _distinct_modes(rng, 25, draw)
    k_f = _distinct_modes(rng, 1, draw, forbid=k_a)
    a0 = 4.0 * float(np.ceil(np.linalg.norm(c)))
    af, ah = _real_from_half(d, k_a, (c / 2).astype(np.complex128), a0=a0)
    ff, fh = _real_from_half(d, k_f, np.array([-0.5j], dtype=np.complex128))
    return Problem(d, af, ah, ff, fh, level=level, name=f"highsparsity/d{d}/N{level}/{instance}")


@dataclasses.dataclass
class AdrProblem:
    """-div(a grad u) + b . grad u + c u = f (Remark ADR).  b_hat[i] holds the d components'
    coefficients at b_freqs[i]; every support is listed with its negation."""
    d: int
    a_freqs: np.ndarray
    a_hat: np.ndarray
    b_freqs: np.ndarray
    b_hat: np.ndarray
    c_freqs: np.ndarray
    c_hat: np.ndarray
    f_freqs: np.ndarray
    f_hat: np.ndarray
    level: int
    name: str = ""

    def union(self) -> np.ndarray:
        """supp(a) u supp(b) u supp(c), closed under negation, with 0 (sorted rows)."""
        pts = {tuple(int(v) for v in w) for fr in (self.a_freqs, self.b_freqs, self.c_freqs) for w in fr}
        pts |= {tuple(-v for v in t) for t in pts}
        pts.add(tuple([0] * self.d))
        return np.array(sorted(pts), dtype=np.int16).reshape(-1, self.d)

    def diffusion_on_union(self) -> Problem:
        """The diffusion problem the stamp and operator are built from: support W = the union,
        a's coefficients on it (0 where a has none)."""
        W = self.union()
        amap = {tuple(int(v) for v in w): c for w, c in zip(self.a_freqs, self.a_hat)}
        ah = np.array([amap.get(tuple(int(v) for v in w), 0.0) for w in W], dtype=np.complex128)
        return Problem(self.d, W, ah, self.f_freqs, self.f_hat, level=self.level, name=self.name)


def _trig(rng, d, n_sin, n_cos, draw, coef, forbid=()):
    """Frequencies and coefficients of sum c sin(2 pi k.x) + sum c cos(2 pi k.x) as a
    conjugate-symmetric list (sin: -i c / 2 at k; cos: c / 2 at k)."""
    modes = _distinct_modes(rng, n_sin + n_cos, draw, forbid)
    c = coef(n_sin + n_cos)
    amps = np.concatenate([-0.5j * c[:n_sin], 0.5 * c[n_sin:]]).astype(np.complex128)
    fr, co = _real_from_half(d, modes, amps)
    return fr, co, c


def adr3d(level: int, instance: int = 0, n_b: int = 5, n_c: int = 5) -> AdrProblem:
    """The exactly sparse 3-D ADR problem of Sec. 10.5 (Eq. ADRTerms): a = a_0 + 2 sine + 2 cosine
    modes, each b_j and c (c with c_0) n_b resp. n_c sine + cosine modes each (the paper: 5 + 5,
    the default), f = 2 sine + 3 cosine modes; every frequency uniform in [-49, 50]^3; a and f
    coefficients U[-1, 1], b and c coefficients U[0, 1]; a_0 = 4 ceil(|c_a|_2), c_0 = 4 ceil(|c_c|_2).
    With the paper's counts the operator has 45 terms and the union support 89 entries."""
    d = 3
    rng = np.random.Generator(np.random.PCG64(9000 + instance))
    draw = lambda: rng.integers(-49, 51, size=d)
    u11 = lambda n: rng.uniform(-1.0, 1.0, size=n)
    u01 = lambda n: rng.uniform(0.0, 1.0, size=n)
    af, ah, ca = _trig(rng, d, 2, 2, draw, u11)
    af = np.concatenate([np.zeros((1, d), dtype=np.int16), af])
    ah = np.concatenate([[4.0 * np.ceil(np.linalg.norm(ca))], ah]).astype(np.complex128)
    bf_list, bh_list = [], []
    for j in range(d):
        fr, co, _ = _trig(rng, d, n_b, n_b, draw, u01)
        bh = np.zeros((len(fr), d), dtype=np.complex128)
        bh[:, j] = co
        bf_list.append(fr)
        bh_list.append(bh)
    # merge the components at shared frequencies
    bmap = {}
    for fr, bh in zip(bf_list, bh_list):
        for w, v in zip(fr, bh):
            t = tuple(int(x) for x in w)
            bmap[t] = bmap.get(t, np.zeros(d, dtype=np.complex128)) + v
    bf = np.array(sorted(bmap), dtype=np.int16).reshape(-1, d)
    bh = np.array([bmap[tuple(int(x) for x in w)] for w in bf], dtype=np.complex128)
    cf, ch, cc = _trig(rng, d, n_c, n_c, draw, u01)
    cf = np.concatenate([np.zeros((1, d), dtype=np.int16), cf])
    ch = np.concatenate([[4.0 * np.ceil(np.linalg.norm(cc))], ch]).astype(np.complex128)
    ff, fh, _ = _trig(rng, d, 2, 3, draw, u11)
    return AdrProblem(d, af, ah, bf, bh, cf, ch, ff, fh, level=level, name=f"adr3d/N{level}/{instance}")


CONFIGS = {1: cfg1, 2: cfg2, 3: cfg3, 4: cfg4}


def make(config: int, instance: int = 0, **kw) -> Problem:
    return CONFIGS[config](instance, **kw) if kw else CONFIGS[config](instance)
