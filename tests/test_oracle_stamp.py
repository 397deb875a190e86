"""Pins for the oracle's stamping set (Sec. 6, Eq. StampSet; App. A).

Each check compares the brute-force Minkowski construction against something
fixed independently of it: hand-derived tiny sets, closed forms for a single
cosine mode and for the tensor-grid coefficient of the multiscale workload,
the App. A count (exact when no sums coincide), nestedness, and an
independent lexicographic sort.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import stamp as ost

Z2 = np.zeros((1, 2), dtype=np.int64)


def _support(*ws):
    """Full symmetric support {0, +-w...}."""
    d = len(ws[0]) if ws else 2
    out = [np.zeros(d, dtype=np.int64)]
    for w in ws:
        out += [np.array(w), -np.array(w)]
    return np.array(out, dtype=np.int64)


def test_tiny_chain_by_hand():
    # F = {(1,0)}, supp a = {0, +-(0,1)}, N = 2: the chain (1, m), |m| <= 2.
    keys, lev = ost.stamp([[1, 0]], _support((0, 1)), 2)
    assert keys.tolist() == [[1, -2], [1, -1], [1, 0], [1, 1], [1, 2]]
    assert lev.tolist() == [2, 1, 0, 1, 2]


def test_tiny_diamond_by_hand():
    # F = {(0,1)}, supp a = {0, +-e1, +-e2}: S^N is the l1 ball of radius N
    # around (0,1); the level is the l1 distance.  N = 2 gives 1 + 4 + 8 = 13.
    keys, lev = ost.stamp([[0, 1]], _support((1, 0), (0, 1)), 2)
    expect = sorted((i, 1 + j) for i in range(-2, 3) for j in range(-2, 3)
                    if abs(i) + abs(j) <= 2)
    assert [tuple(k) for k in keys.tolist()] == expect
    assert lev.tolist() == [abs(k[0]) + abs(k[1] - 1) for k in expect]
    assert len(keys) == ost.cardinality_bound(1, 5, 2) == 13


def _generic_instance(rng, d, half, n_f, spread=10 ** 4):
    """Random frequencies so large and spread that no two sums coincide."""
    A = rng.integers(-spread, spread, size=(half, d))
    F = rng.integers(-spread, spread, size=(n_f, d))
    return F, np.concatenate([np.zeros((1, d), dtype=np.int64), A, -A])


@pytest.mark.parametrize("d,half,n_f,N", [(40, 5, 6, 3), (3, 4, 3, 3), (10, 10, 4, 2), (7, 2, 5, 4)])
def test_app_a_count_is_exact_in_generic_position(d, half, n_f, N):
    rng = np.random.default_rng(1000 + d)
    F, A = _generic_instance(rng, d, half, n_f)
    keys, lev = ost.stamp(F, A, N)
    s = 2 * half + 1
    assert len(keys) == ost.cardinality_bound(n_f, s, N)
    # and level by level: the level-n shell has |F| sum_t 2^t C(|A|,t) C(n-1,t-1)
    for n in range(N + 1):
        shell = ost.cardinality_bound(n_f, s, n) - (ost.cardinality_bound(n_f, s, n - 1) if n else 0)
        assert int((lev == n).sum()) == shell


def test_app_a_count_worked_case():
    # d = 40, |A| = 5, |F| = 6, N = 3 -> 1386 by the count
    assert ost.cardinality_bound(6, 11, 3) == 6 * (1 + 10 + (10 + 40) + (10 + 80 + 80))


@pytest.mark.parametrize("seed", range(4))
def test_app_a_count_bounds_low_dim(seed):
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, size=(3, 2))
    A = A[np.any(A != 0, axis=1)]
    sup = {tuple(w) for w in A} | {tuple(-w) for w in A} | {(0, 0)}
    F = np.unique(rng.integers(-5, 6, size=(4, 2)), axis=0)
    keys, _ = ost.stamp(F, np.array(sorted(sup)), 3)
    assert len(keys) <= ost.cardinality_bound(len(F), len(sup), 3)


def test_single_mode_closed_form():
    # supp a = {0, +-w}: S^N = F + {m w : |m| <= N} with level |m|.
    rng = np.random.default_rng(7)
    d, N = 6, 4
    w = rng.integers(-50, 50, size=d)
    F = rng.integers(-1000, 1000, size=(5, d))
    keys, lev = ost.stamp(F, _support(tuple(w)), N)
    expect = {}
    for f in F:
        for m in range(-N, N + 1):
            k = tuple(int(v) for v in f + m * w)
            expect[k] = min(expect.get(k, N + 1), abs(m))
    assert len(keys) == len(F) * (2 * N + 1) == len(expect)
    assert {tuple(k): int(l) for k, l in zip(keys.tolist(), lev)} == expect


def test_multiscale_grid_closed_form():
    # a = prod_j (1 + 0.5 sin(2 pi K_j x_j)), K = (1, 32, 512): supp a is the
    # tensor grid {(i, 32 j, 512 l) : |i|,|j|,|l| <= 1}; one stamp moves each
    # index by at most one, so S^N = F + {(i, 32j, 512l) : max(|i|,|j|,|l|) <= N}
    # with level = the smallest such max over representations.
    rng = np.random.default_rng(3)
    grid = np.array([(i, 32 * j, 512 * l) for i in (-1, 0, 1) for j in (-1, 0, 1) for l in (-1, 0, 1)])
    F = rng.integers(-64, 65, size=(6, 3))
    N = 3
    keys, lev = ost.stamp(F, grid, N)
    expect = {}
    for f in F:
        for i, j, l in itertools.product(range(-N, N + 1), repeat=3):
            k = (int(f[0] + i), int(f[1] + 32 * j), int(f[2] + 512 * l))
            expect[k] = min(expect.get(k, N + 1), max(abs(i), abs(j), abs(l)))
    assert {tuple(k): int(v) for k, v in zip(keys.tolist(), lev)} == expect


def test_nested_and_levels_first_appearance():
    rng = np.random.default_rng(11)
    F = rng.integers(-4, 5, size=(3, 2))
    F = np.unique(F, axis=0)
    A = _support((1, 2), (-2, 1), (0, 3))
    sets = ost.stamp_sets(F, A, 3)
    for n in range(1, 4):
        assert sets[n - 1] <= sets[n]           # 0 in supp(a)
    keys, lev = ost.stamp(F, A, 3)
    for k, l in zip(keys.tolist(), lev):
        k = tuple(k)
        assert k in sets[l] and (l == 0 or k not in sets[l - 1])


def test_lex_order_matches_numpy_lexsort():
    rng = np.random.default_rng(5)
    F, A = _generic_instance(rng, 5, 3, 4, spread=20)
    keys, _ = ost.stamp(F, A, 2)
    order = np.lexsort(keys.T[::-1])          # last key is primary -> coordinate 0
    assert np.array_equal(order, np.arange(len(keys)))
    assert len(np.unique(keys, axis=0)) == len(keys)


def test_canonical_a_completion_and_errors():
    freqs = np.array([[0, 0], [1, 2], [3, -1]])
    coef = np.array([2.0, 0.1 + 0.2j, 0.05j])
    f, c = ost.canonical_a(freqs, coef)
    assert [tuple(x) for x in f.tolist()] == [(-3, 1), (-1, -2), (0, 0), (1, 2), (3, -1)]
    assert np.allclose(c, [-0.05j, 0.1 - 0.2j, 2.0, 0.1 + 0.2j, 0.05j])
    with pytest.raises(ost.OracleInputError):
        ost.canonical_a(np.array([[0, 0], [1, 0], [-1, 0]]), np.array([1.0, 0.1, 0.2]))
    with pytest.raises(ost.OracleInputError):
        ost.canonical_a(np.array([[1, 0]]), np.array([0.1]))       # no a_0
    f, c = ost.canonical_a(np.array([[0, 0], [1, 0], [2, 0]]), np.array([1.0, 0.0, 0.1]))
    assert [tuple(x) for x in f.tolist()] == [(-2, 0), (0, 0), (2, 0)]   # zero dropped
