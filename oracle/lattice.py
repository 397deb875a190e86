"""Oracle: random rank-1 lattices as a map of frequency sets (Sec. 8, Definition of a
reconstructing rank-1 lattice, Lemma RandomRank1Lattice).

Test infrastructure only: plain, exact integer arithmetic, no blocking or reordering.

* ``lattice_values(keys, z, M)``: the lattice value ``k . z mod M`` of every frequency k (the
  index of k in the length-M one-dimensional transform along the lattice).
* ``is_reconstructing(keys, z, M)``: the Definition -- distinct frequencies of the set have
  distinct lattice values.
* ``expansion(keys)``: K of the Lemma, the side of the smallest cube holding the set.
* ``next_prime(x)``: the smallest prime greater than x, by trial division.
* ``lemma_modulus(keys, sigma)``: the Lemma's M, the smallest prime above max(K, |I|^2 / sigma).

Pins (tests/test_oracle_lattice.py): known primes; the proof's criterion (no difference k - l
of the set is orthogonal to z modulo M) checked pair by pair against the Definition; d = 1,
where every z works once M is a prime above K; a set larger than M, which no lattice of M points
can reconstruct; and the Lemma's failure probability, at most sigma, on repeated draws.
"""
import math

import numpy as np


def lattice_values(keys, z, M):
    """k . z mod M for every row k of keys [n x d] (Definition of the rank-1 lattice: the
    lattice point j / M z pairs with frequency k through the exponent k . z j / M)."""
    keys = np.asarray(keys, dtype=np.int64)
    z = [int(v) for v in z]
    M = int(M)
    out = np.empty(len(keys), dtype=np.int64)
    for r in range(len(keys)):
        out[r] = sum(int(keys[r, i]) * z[i] for i in range(keys.shape[1])) % M
    return out


def is_reconstructing(keys, z, M):
    """Definition: k . z and l . z differ modulo M for every pair of distinct k, l of the set."""
    uniq = {tuple(int(v) for v in k) for k in np.asarray(keys)}
    vals = lattice_values(np.array(sorted(uniq), dtype=np.int64).reshape(len(uniq), -1), z, M)
    return len(set(vals.tolist())) == len(uniq)


def expansion(keys):
    """K of the Lemma: max over coordinates of (largest minus smallest entry in the set)."""
    keys = np.asarray(keys, dtype=np.int64)
    return int((keys.max(axis=0) - keys.min(axis=0)).max())


def next_prime(x):
    """Smallest prime strictly greater than x (trial division by every odd number up to the root)."""
    p = max(2, math.floor(x) + 1)
    while True:
        if p == 2 or (p % 2 and all(p % q for q in range(3, math.isqrt(p) + 1, 2))):
            return p
        p += 1


def lemma_modulus(keys, sigma):
    """Lemma RandomRank1Lattice: M is the smallest prime greater than max(K, |I|^2 / sigma)."""
    n = len({tuple(int(v) for v in k) for k in np.asarray(keys)})
    return next_prime(max(expansion(keys), n * n / sigma))
