"""Host logic of the rank-1 lattice entry points (no device work): the Lemma's modulus from
ss_lattice_modulus against the oracle's trial-division prime search, and its argument errors."""
import numpy as np
import pytest

from oracle import lattice as ol


@pytest.fixture(scope="module")
def ss():
    from paper_2302_00752_amd import sparsespec
    return sparsespec


@pytest.mark.parametrize("K,n,sigma", [(0, 0, 1.0), (40, 0, 1.0), (40, 3, 1.0), (1, 10, 0.1), (64, 31220, 0.01),
                                       (32766, 1000, 0.5), (10, 2, 0.3), (0, 7, 1.0)])
def test_modulus_matches_oracle(ss, K, n, sigma):
    assert ss.lattice_modulus(K, n, sigma) == ol.next_prime(max(K, n * n / sigma))


def test_modulus_of_a_set_matches_the_lemma(ss):
    rng = np.random.default_rng(21)
    keys = np.unique(rng.integers(-9, 10, size=(200, 4)), axis=0)
    assert ss.lattice_modulus(ol.expansion(keys), len(keys), 0.05) == ol.lemma_modulus(keys, 0.05)


def test_modulus_errors(ss):
    for args in ((5, 5, 0.0), (5, 5, 1.5), (-1, 5, 0.5), (5, -1, 0.5)):
        with pytest.raises(ss.SparseSpecError) as e:
            ss.lattice_modulus(*args)
        assert e.value.status == ss.SS_EINVAL, args
    with pytest.raises(ss.SparseSpecError) as e:
        ss.lattice_modulus(0, 1 << 21, 0.5)          # n^2 / sigma = 2^43 > 2^40
    assert e.value.status == ss.SS_ERANGE
