"""The truncated Galerkin operator and its direct solve (oracle; tests only).

* ``neighbours``   for each k in S^N and each w in supp(a) (lexicographic
                   a-table order): the slot of l = k - w if l is in S^N.  Sec.
                   9, Eq. FiniteGalerkinOperator sums over l in S^N only, and
                   a_{k-l} vanishes unless k - l is in supp(a).
* ``classes``      connected classes of that relation (Sec. 6, proof of Prop.
                   SolutionSupport: the system splits into one independent
                   block per class).  Class id = smallest slot in the class.
* ``matrix``       the entries 4 pi^2 (k . l) a_{k-l} of L_N (Alg. 1, step 4),
                   with the dot product k . l formed directly in exact
                   integers, stored as a scipy sparse matrix.
* ``apply``        y = L_N x.
* ``proxy_error``  the relative proxy error |f - L u^N|_2 / |f|_2 of Sec. 10.1
                   (Lemma ProxyError), with L the untruncated operator: every
                   term 4 pi^2 (k . l) a_{k-l} u_l for l in S^N and k - l in
                   supp(a) is summed at its k (Prop. LExpansion: L u^N lives
                   on S^N + supp(a) = S^{N+1}), so the l2 norm is exact.
* ``solve``        the mean-zero solution of L_N u = f on S^N (Alg. 1, step 5):
                   one dense complex LU solve per class; the row and column of
                   k = 0 vanish identically and u_0 = 0 (Sec. 3, space H;
                   Prop. ExistenceUniquenessStability needs f_0 = 0).  A class
                   larger than ``dense_limit`` is solved by textbook
                   Jacobi-preconditioned CG in float64 instead.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp

FOUR_PI2 = 4.0 * np.pi ** 2


def slot_index(keys) -> Dict[Tuple[int, ...], int]:
    return {tuple(int(v) for v in k): i for i, k in enumerate(np.asarray(keys))}


def _byte_index(keys) -> Dict[bytes, int]:
    """Slot of each key, keyed by the raw bytes of its int64 coordinates."""
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    return {keys[i].tobytes(): i for i in range(len(keys))}


def neighbours(keys, a_freqs):
    """Canonical CSR of the neighbour relation in (row, a-table index) order.

    Returns ``(row_ptr [n+1], cols [nnz], js [nnz])``, all int64.
    """
    keys = np.asarray(keys, dtype=np.int64)
    a_freqs = np.asarray(a_freqs, dtype=np.int64)
    index = _byte_index(keys)
    n, s = len(keys), len(a_freqs)
    col = np.full((n, s), -1, dtype=np.int64)
    for j, w in enumerate(a_freqs):
        shifted = np.ascontiguousarray(keys - w)
        for i in range(n):
            m = index.get(shifted[i].tobytes())
            if m is not None:
                col[i, j] = m
    present = col >= 0
    row_ptr = np.concatenate([[0], np.cumsum(present.sum(axis=1))]).astype(np.int64)
    jj = np.broadcast_to(np.arange(s, dtype=np.int64), (n, s))
    return row_ptr, col[present], jj[present].copy()


def classes(row_ptr, cols):
    """Connected-class label of each slot: the smallest slot of its class."""
    n = len(row_ptr) - 1
    label = np.full(n, -1, dtype=np.int64)
    for start in range(n):
        if label[start] >= 0:
            continue
        label[start] = start
        stack = [start]
        while stack:
            i = stack.pop()
            for m in cols[row_ptr[i]:row_ptr[i + 1]]:
                if label[m] < 0:
                    label[m] = start
                    stack.append(m)
    return label


def matrix(keys, a_freqs, a_hat, nbr=None):
    """L_N as a sparse complex128 matrix, entries by the definition.

    ``nbr`` may pass a precomputed ``neighbours(keys, a_freqs)``.
    """
    keys = np.asarray(keys, dtype=np.int64)
    a_hat = np.asarray(a_hat, dtype=np.complex128)
    row_ptr, cols, js = neighbours(keys, a_freqs) if nbr is None else nbr
    rows = np.repeat(np.arange(len(keys)), np.diff(row_ptr))
    k_dot_l = np.einsum("ij,ij->i", keys[rows], keys[cols])   # exact int64
    vals = FOUR_PI2 * k_dot_l.astype(np.float64) * a_hat[js]
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(keys), len(keys)))


def apply(keys, a_freqs, a_hat, x):
    """y = L_N x on S^N."""
    return matrix(keys, a_freqs, a_hat) @ np.asarray(x, dtype=np.complex128)


def proxy_error(keys, u, a_freqs, a_hat, f_freqs, f_hat):
    """|f - L u|_2 / |f|_2 for u given on the keys (Sec. 10.1, Lemma ProxyError).

    L u is formed term by term without truncation: each (l, w) pair, l a key
    and w in supp(a), adds 4 pi^2 (k . l) a_w u_l at k = l + w.  Terms are
    gathered per distinct k; f enters at its own frequencies.
    """
    keys = np.asarray(keys, dtype=np.int64)
    u = np.asarray(u, dtype=np.complex128)
    a_freqs = np.asarray(a_freqs, dtype=np.int64)
    a_hat = np.asarray(a_hat, dtype=np.complex128)
    f_freqs = np.asarray(f_freqs, dtype=np.int64)
    f_hat = np.asarray(f_hat, dtype=np.complex128)
    n, s, d = len(keys), len(a_freqs), keys.shape[1]
    k = (keys[:, None, :] + a_freqs[None, :, :]).reshape(n * s, d)       # k = l + w
    l = np.repeat(keys, s, axis=0)
    k_dot_l = np.einsum("ij,ij->i", k, l)                                  # exact int64
    terms = FOUR_PI2 * k_dot_l.astype(np.float64) * np.tile(a_hat, n) * np.repeat(u, s)
    allk = np.concatenate([k, f_freqs])
    vals = np.concatenate([-terms, f_hat])                                 # f - L u
    uniq, inv = np.unique(allk, axis=0, return_inverse=True)
    res = np.zeros(len(uniq), dtype=np.complex128)
    np.add.at(res, inv.ravel(), vals)
    return float(np.linalg.norm(res) / np.linalg.norm(f_hat))


def _pcg(M, f, D, tol=1e-15, max_iter=100000):
    """Textbook Jacobi-preconditioned conjugate gradients, float64."""
    x = np.zeros_like(f)
    r = f.copy()
    z = r / D
    p = z.copy()
    rho = np.vdot(r, z).real
    fn = np.linalg.norm(f)
    for _ in range(max_iter):
        if np.linalg.norm(r) <= tol * fn:
            break
        q = M @ p
        alpha = rho / np.vdot(p, q).real
        x += alpha * p
        r -= alpha * q
        z = r / D
        rho_new = np.vdot(r, z).real
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


def solve(keys, a_freqs, a_hat, f, dense_limit: int = 6000, M=None):
    """Mean-zero solution of L_N u = f on S^N (Alg. 1, steps 4-5, per class)."""
    keys = np.asarray(keys, dtype=np.int64)
    f = np.asarray(f, dtype=np.complex128)
    nbr = neighbours(keys, a_freqs)
    label = classes(nbr[0], nbr[1])
    if M is None:
        M = matrix(keys, a_freqs, a_hat, nbr)
    M = sp.csr_matrix(M)
    u = np.zeros(len(keys), dtype=np.complex128)
    nonzero_k = np.any(keys != 0, axis=1)
    if np.any(f[~nonzero_k] != 0):
        raise ValueError("f_0 must vanish (mean-zero forcing)")
    for c in np.unique(label):
        rows = np.nonzero((label == c) & nonzero_k)[0]
        if len(rows) == 0:
            continue
        block = M[rows][:, rows]
        if len(rows) <= dense_limit:
            u[rows] = np.linalg.solve(block.toarray(), f[rows])
        else:
            u[rows] = _pcg(block, f[rows], np.real(block.diagonal()))
    return u
