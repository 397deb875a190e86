"""Advection-diffusion-reaction extension of the Galerkin system (oracle; tests only).

The problem -div(a grad u) + b . grad u + c u = f on the d-torus (Remark ADR, Eq. ADR).
With e_k(x) = exp(2 pi i k.x) and grad e_l = 2 pi i l e_l, the Fourier coefficient at k of
each term applied to u = sum_l u_l e_l is

    diffusion   sum_l 4 pi^2 (k . l) a_{k-l} u_l
    advection   sum_l 2 pi i (l . b_{k-l}) u_l          (b_w = (b_{1,w}, ..., b_{d,w}))
    reaction    sum_l c_{k-l} u_l

so the truncated operator on a set S has entries
L_{k,l} = 4 pi^2 (k.l) a_{k-l} + 2 pi i (l . b_{k-l}) + c_{k-l} for k, l in S.

* ``support``   the union of supp(a), supp(b_j) and supp(c), closed under negation, with 0: the
                set the stamp adds per level (reading: one application of the operator shifts a
                frequency by one element of one of the supports, so S^N = S^{N-1} + union is
                the smallest set holding the operator's N-fold action on F).
* ``matrix``    L on a key set, entry by entry from the definition above, exact integer dot
                products.
* ``solve``     L u = f on the key set, one direct solve per connected class (the relation is
                still the union-support shift, so classes still decouple): a dense LU up to
                ``dense_limit`` rows, a sparse LU (SuperLU) of the same block above (the paper's
                3-D data at level 2 form one class of about 4e4 rows).  The reaction term's
                c_0 > 0 keeps the zero frequency an ordinary unknown.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import galerkin as og
from oracle import stamp as ost

FOUR_PI2 = 4.0 * np.pi ** 2
TWO_PI = 2.0 * np.pi


def _table(freqs, coef, width=None) -> Dict[Tuple[int, ...], np.ndarray]:
    out: Dict[Tuple[int, ...], np.ndarray] = {}
    for w, c in zip(np.asarray(freqs, dtype=np.int64), coef):
        t = tuple(int(v) for v in w)
        if t in out:
            raise ost.OracleInputError(f"duplicate frequency {t}")
        out[t] = np.asarray(c, dtype=np.complex128).reshape(-1 if width is None else width)
    return out


def support(a_freqs, b_freqs, c_freqs, d: int) -> np.ndarray:
    """supp(a) u supp(b) u supp(c), closed under negation, with 0, in lexicographic order."""
    pts = set()
    for fr in (a_freqs, b_freqs, c_freqs):
        for w in np.asarray(fr, dtype=np.int64).reshape(-1, d):
            t = tuple(int(v) for v in w)
            pts.add(t)
            pts.add(tuple(-v for v in t))
    pts.add(tuple([0] * d))
    return np.array(ost.lex_sort(list(pts)), dtype=np.int64).reshape(-1, d)


def matrix(keys, a_freqs, a_hat, b_freqs, b_hat, c_freqs, c_hat):
    """L on the key set as a scipy sparse complex128 matrix (entries by the definition).

    b_hat[i] is the d-vector (b_{1,w}, ..., b_{d,w}) at b_freqs[i].
    """
    keys = np.asarray(keys, dtype=np.int64)
    n, d = keys.shape
    A = _table(a_freqs, a_hat, 1)
    B = _table(b_freqs, b_hat, d)
    Cc = _table(c_freqs, c_hat, 1)
    W = support(a_freqs, b_freqs, c_freqs, d)
    pos = og.slot_index(keys)
    rows, cols, vals = [], [], []
    for w in W:
        t = tuple(int(v) for v in w)
        aw = A[t][0] if t in A else 0.0
        bw = B[t] if t in B else np.zeros(d, dtype=np.complex128)
        cw = Cc[t][0] if t in Cc else 0.0
        for i in range(n):
            l = keys[i] - w
            m = pos.get(tuple(int(v) for v in l))
            if m is None:
                continue
            k = keys[i]
            v = FOUR_PI2 * float(int(np.dot(k, l))) * aw + TWO_PI * 1j * np.dot(l.astype(np.float64), bw) + cw
            rows.append(i)
            cols.append(m)
            vals.append(v)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(n, n))


def solve(keys, a_freqs, a_hat, b_freqs, b_hat, c_freqs, c_hat, f, M=None, dense_limit: int = 6000):
    """u with L u = f on the key set: one LU solve per connected class (dense up to
    ``dense_limit`` rows, sparse above)."""
    keys = np.asarray(keys, dtype=np.int64)
    d = keys.shape[1]
    if M is None:
        M = matrix(keys, a_freqs, a_hat, b_freqs, b_hat, c_freqs, c_hat)
    M = sp.csr_matrix(M)
    W = support(a_freqs, b_freqs, c_freqs, d)
    row_ptr, cols, _ = og.neighbours(keys, W)
    label = og.classes(row_ptr, cols)
    f = np.asarray(f, dtype=np.complex128)
    u = np.zeros(len(keys), dtype=np.complex128)
    for c in np.unique(label):
        rows = np.nonzero(label == c)[0]
        block = M[rows][:, rows]
        if len(rows) <= dense_limit:
            u[rows] = np.linalg.solve(block.toarray(), f[rows])
        else:
            u[rows] = spla.spsolve(sp.csc_matrix(block), f[rows])
    return u
