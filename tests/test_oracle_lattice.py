"""Pins of the rank-1 lattice oracle (Sec. 8: Definition of a reconstructing rank-1 lattice,
Lemma RandomRank1Lattice) against facts that do not come from the oracle itself."""
import itertools

import numpy as np

from oracle import lattice as ol


def test_next_prime_known_values():
    # primes from number-theory tables: 2^31 + 11 is the first prime above 2^31, 10^6 + 3 above 10^6
    assert [ol.next_prime(x) for x in (0, 1, 2, 13, 100, 7918)] == [2, 2, 3, 17, 101, 7919]
    assert ol.next_prime(10 ** 6) == 1000003
    assert ol.next_prime(2 ** 31) == 2147483659
    assert ol.next_prime(99.5) == 101 and ol.next_prime(100.0) == 101


def test_definition_matches_the_proofs_difference_criterion():
    # the proof of the Lemma: reconstructing iff no difference k - l (k != l in I) has
    # (k - l) . z = 0 mod M; checked pair by pair on small sets and many z
    rng = np.random.default_rng(11)
    for trial in range(60):
        d = int(rng.integers(1, 4))
        n = int(rng.integers(2, 9))
        keys = rng.integers(-4, 5, size=(n, d))
        keys = np.unique(keys, axis=0)
        M = int(rng.choice([5, 7, 11, 13, 31]))
        z = rng.integers(1, M, size=d)
        by_pairs = all(int(np.dot(np.subtract(k, l), z)) % M != 0 for k, l in itertools.combinations(keys.tolist(), 2))
        assert ol.is_reconstructing(keys, z, M) == by_pairs, (keys, z, M)


def test_values_are_linear_and_in_range():
    # k . z mod M is a homomorphism Z^d -> Z_M: (k - w) . z = k . z - w . z (mod M)
    rng = np.random.default_rng(12)
    M = 1000003
    z = rng.integers(1, M, size=5)
    k = rng.integers(-300, 300, size=(50, 5))
    w = rng.integers(-300, 300, size=(1, 5))
    hk, hw, hkw = ol.lattice_values(k, z, M), ol.lattice_values(w, z, M), ol.lattice_values(k - w, z, M)
    assert np.all((0 <= hk) & (hk < M))
    assert np.array_equal(hkw, (hk - hw[0]) % M)
    # one coordinate: k z mod M with the arithmetic written out for a worked value
    assert ol.lattice_values(np.array([[-3, 2]]), [5, 7], 11)[0] == (-15 + 14) % 11 == 10


def test_one_dimension_every_z_reconstructs_above_the_expansion():
    # d = 1: k z = l z mod M with M prime > K forces M | (k - l) z, impossible for 0 < |k - l| <= K
    keys = np.arange(-20, 21).reshape(-1, 1)
    K = ol.expansion(keys)
    assert K == 40
    M = ol.next_prime(K)
    assert all(ol.is_reconstructing(keys, [z], M) for z in range(1, M))
    # a modulus below the expansion fails for z = 1 (k and k + M collide)
    assert not ol.is_reconstructing(keys, [1], 37)


def test_more_frequencies_than_lattice_points_never_reconstruct():
    # pigeonhole: M values cannot separate more than M frequencies
    keys = np.array(list(itertools.product(range(4), repeat=2)))   # 16 frequencies
    for z in itertools.product(range(1, 13), repeat=2):
        assert not ol.is_reconstructing(keys, z, 13)


def test_lemma_failure_rate_at_most_sigma():
    # Lemma: z drawn uniformly from {1..M-1}^d with M the smallest prime above max(K, |I|^2/sigma)
    # reconstructs I with probability at least 1 - sigma
    rng = np.random.default_rng(13)
    keys = np.unique(rng.integers(-6, 7, size=(30, 3)), axis=0)
    sigma = 0.5
    M = ol.lemma_modulus(keys, sigma)
    n = len(keys)
    assert M > n * n / sigma and M == ol.next_prime(max(ol.expansion(keys), n * n / sigma))
    fails = sum(not ol.is_reconstructing(keys, rng.integers(1, M, size=3), M) for _ in range(400))
    # the union bound gives at most sigma; the binomial spread of 400 draws is below 0.05
    assert fails / 400 <= sigma
    # a modulus far below |I|^2 fails most of the time (birthday collisions), so the test has teeth
    Msmall = ol.next_prime(n)
    fails_small = sum(not ol.is_reconstructing(keys, rng.integers(1, Msmall, size=3), Msmall) for _ in range(200))
    assert fails_small / 200 > 0.8
