"""Stamping sets, by the definition (oracle; test infrastructure only).

* ``canonical_a``   Sec. 6, proof of Prop. SolutionSupport: a real, positive
                    diffusion coefficient has a support symmetric under
                    negation that contains 0, with conjugate coefficients at
                    +-w.  Half lists are completed with conjugates.
* ``stamp_levels``  Sec. 6, Eq. StampSet: S^0 = F, S^N = S^{N-1} + supp(a)
                    (Minkowski sum), formed in full at every level -- no
                    frontier shortcut.  The level of k is the first n with
                    k in S^n.
* ``lex_sort``      the slot order: ascending lexicographic order on signed
                    integer tuples, coordinate 0 most significant.
* ``cardinality_bound``  App. A, Lemma StampSetCardinality (Eq.
                    CombinatorialStampSetCardinality); equality holds when no
                    two sums coincide.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np


class OracleInputError(ValueError):
    pass


def canonical_a(a_freqs, a_hat, rel_tol: float = 1e-14):
    """Close supp(a) under negation and return it in lexicographic order.

    Returns ``(freqs [s,d] int64, coef [s] complex128)``.  Exact-zero
    coefficients are dropped; a missing -w receives conj(a_w); a present pair
    must be conjugate to ``rel_tol * max|a|``; the coefficient at 0 must be
    real and positive.
    """
    a_freqs = np.asarray(a_freqs, dtype=np.int64)
    a_hat = np.asarray(a_hat, dtype=np.complex128)
    table: Dict[Tuple[int, ...], complex] = {}
    for w, c in zip(a_freqs, a_hat):
        t = tuple(int(v) for v in w)
        if t in table:
            raise OracleInputError(f"duplicate frequency {t}")
        table[t] = complex(c)
    scale = max(abs(c) for c in table.values())
    for t, c in list(table.items()):
        nt = tuple(-v for v in t)
        if nt not in table:
            table[nt] = c.conjugate()
        elif abs(table[nt] - c.conjugate()) > rel_tol * scale:
            raise OracleInputError(f"coefficients at {t} and {nt} are not conjugate")
    table = {t: c for t, c in table.items() if c != 0}
    zero = tuple([0] * a_freqs.shape[1])
    if zero not in table or table[zero].imag != 0 or table[zero].real <= 0:
        raise OracleInputError("a_0 must be real and positive")
    keys = lex_sort(list(table.keys()))
    freqs = np.array(keys, dtype=np.int64).reshape(len(keys), a_freqs.shape[1])
    coef = np.array([table[t] for t in keys], dtype=np.complex128)
    return freqs, coef


def lex_sort(tuples: List[Tuple[int, ...]]) -> List[Tuple[int, ...]]:
    """Ascending lexicographic order of integer tuples (Python tuple order)."""
    return sorted(tuples)


def stamp_levels(F, a_support, N: int) -> Dict[Tuple[int, ...], int]:
    """Map every k in S^N[a](F) to its level: the first n with k in S^n."""
    F = [tuple(int(v) for v in k) for k in np.asarray(F, dtype=np.int64)]
    if len(set(F)) != len(F):
        raise OracleInputError("duplicate forcing frequency")
    A = [tuple(int(v) for v in w) for w in np.asarray(a_support, dtype=np.int64)]
    level: Dict[Tuple[int, ...], int] = {k: 0 for k in F}
    S_prev = set(F)
    for n in range(1, N + 1):
        S_n = set()
        for k in S_prev:                       # the whole previous set
            for w in A:
                S_n.add(tuple(ki + wi for ki, wi in zip(k, w)))
        for k in S_n:
            if k not in level:
                level[k] = n
        S_prev = S_n
    return level


def stamp(F, a_support, N: int):
    """S^N in slot order: ``(keys [n,d] int64, levels [n] int64)``."""
    level = stamp_levels(F, a_support, N)
    keys = lex_sort(list(level.keys()))
    d = np.asarray(F).shape[1]
    return (np.array(keys, dtype=np.int64).reshape(len(keys), d),
            np.array([level[k] for k in keys], dtype=np.int64))


def stamp_sets(F, a_support, N: int) -> List[set]:
    """All of S^0, ..., S^N as Python sets (for nestedness checks)."""
    F = [tuple(int(v) for v in k) for k in np.asarray(F, dtype=np.int64)]
    A = [tuple(int(v) for v in w) for w in np.asarray(a_support, dtype=np.int64)]
    out = [set(F)]
    for _ in range(N):
        out.append({tuple(ki + wi for ki, wi in zip(k, w)) for k in out[-1] for w in A})
    return out


def cardinality_bound(n_f: int, s: int, N: int) -> int:
    """App. A bound |F| sum_{n<=N} sum_t 2^t C(|A|,t) C(n-1,t-1), |A| = (s-1)/2.

    The binomial C(n-1, t-1) at n = t = 0 is read as 1, so that level 0
    contributes |F|.
    """
    half = (s - 1) // 2

    def c(n, k):
        if n == -1 and k == -1:
            return 1
        if n < 0 or k < 0 or k > n:
            return 0
        return math.comb(n, k)

    return n_f * sum(2 ** t * c(half, t) * c(n - 1, t - 1)
                     for n in range(N + 1) for t in range(0, min(n, half) + 1))
