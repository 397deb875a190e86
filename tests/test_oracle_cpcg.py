"""The timed CPU baseline (oracle/cpcg.c, sparse FP64 Jacobi PCG in C) against the pinned oracle:
its stamp sizes equal the brute-force stamp's, its solutions the per-class dense solve's (which the
other oracle tests pin to the paper), the constant-coefficient case the Poisson closed form, and
one thread or several give the same answers."""
import numpy as np
import pytest

from oracle import cpcg
from oracle import galerkin as og
from oracle import stamp as ost
from paper_2302_00752_amd import workloads


def _oracle(p):
    af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
    keys, _ = ost.stamp(p.f_freqs, af, p.level)
    pos = og.slot_index(keys)
    f = np.zeros(len(keys), dtype=np.complex128)
    for k, v in zip(p.f_freqs, p.f_hat):
        f[pos[tuple(int(x) for x in k)]] = v
    return keys, og.solve(keys, af, ah, f)


@pytest.mark.parametrize("case", [(1, 0, None), (1, 3, None), (2, 0, 2), (3, 0, 2), (4, 0, 1)])
def test_matches_dense_oracle(case):
    config, inst, level = case
    p = workloads.make(config, inst) if level is None else workloads.make(config, inst, level=level)
    keys, uo = _oracle(p)
    st, info, used, u = cpcg.solve_batch([p], 1e-13, threads=1, want_u=True)
    assert st == 0 and info[0]["n"] == len(keys) and info[0]["rel_residual"] <= 1e-12
    assert np.linalg.norm(u[0] - uo) / np.linalg.norm(uo) <= 1e-10


def test_poisson_closed_form_and_threads():
    # supp(a) = {0}: u_k = f_k / (4 pi^2 |k|^2 a_0), in canonical (lexicographic) order
    fq = np.array([[1, 2, 3], [-1, -2, -3], [4, 0, 0]], dtype=np.int16)
    fh = np.array([1 + 1j, 1 - 1j, 0.5])
    p = workloads.Problem(d=3, a_freqs=np.zeros((1, 3), np.int16), a_hat=np.array([2.0 + 0j]), f_freqs=fq,
                          f_hat=fh, level=2)
    st, info, _, u = cpcg.solve_batch([p], 1e-14, threads=1, want_u=True)
    order = np.lexsort(fq.T[::-1])
    closed = fh[order] / (4 * np.pi ** 2 * 2.0 * (fq[order].astype(np.int64) ** 2).sum(1))
    assert st == 0 and np.allclose(u[0], closed, rtol=1e-13, atol=0)
    probs = [workloads.make(2, i, level=2) for i in range(6)]
    s1, i1, n1, u1 = cpcg.solve_batch(probs, 1e-10, threads=1, want_u=True)
    s4, i4, n4, u4 = cpcg.solve_batch(probs, 1e-10, threads=4, want_u=True)
    assert n1 == 1 and n4 == 4 and s1 == s4 == 0
    for a, b in zip(u1, u4):
        assert np.array_equal(a, b)
    assert all(x["n"] == workloads.generic_stamp_size(20, 21, 2) for x in i1)
