"""Pins of the oracle's summation-depth shift (the shift-policy question of the remark after
Table 3 and of Section 8): a Gram summed in chunks of c rows has summation depth
d = c + ceil(m / c), its error obeys the gamma_d bound of Section 3.1.1 in place of gamma_m, and
the shift s = 11 (d n + n (n+1)) u ||X||_2^2 reduces to equation (eq:finds2) at d = m.
"""
from fractions import Fraction

import numpy as np
import pytest

import accuracy
import oracle
import synth

U = 2.0 ** -53


def test_chunked_gram_exact_on_integers():
    # small integer entries: every product and partial sum is exact, for any summation order
    rng = np.random.default_rng(3)
    X = rng.integers(-9, 10, size=(997, 13)).astype(float)
    A = oracle.gram(X)
    for c in (1, 2, 7, 64, 500, 997, 5000):
        np.testing.assert_array_equal(oracle.gram_chunked(X, c), A)
    np.testing.assert_array_equal(A, X.T @ X)


@pytest.mark.parametrize("chunk,expect", [(1, 1.0), (2, 1.0), (3, 1.0 + 2.0 ** -51),
                                          (4, 1.0 + 2.0 ** -52), (8, 1.0), (9, 1.0)])
def test_chunk_boundaries_decide_the_rounding(chunk, expect):
    # one column x = (1, 2^-27 x 8): the squares are 1 and eight times 2^-54, exact sum
    # 1 + 2^-51.  Added one by one to 1 every 2^-54 is lost (row-order sum: 1); summed first in
    # chunks they survive in part, and where they land is fixed by the chunk boundaries and by
    # adding the chunk sums in chunk order (round to nearest even on the ties).
    x = np.array([[1.0]] + [[2.0 ** -27]] * 8)
    assert oracle.gram(x)[0, 0] == 1.0
    assert oracle.gram_chunked(x, chunk)[0, 0] == expect


def test_depth_closed_form():
    assert oracle.gram_depth(1000, 37) == 37 + 28
    assert oracle.gram_depth(1000, 1) == 1 + 1000
    assert oracle.gram_depth(1000, 1000) == 1000
    assert oracle.gram_depth(1000, 4096) == 1000
    assert oracle.gram_depth(4096, 64) == 128


@pytest.mark.parametrize("m,n,chunk", [(3000, 4, 50), (2048, 3, 1), (1500, 5, 1500)])
def test_chunked_gram_within_gamma_depth(m, n, chunk):
    # |A - X^T X| <= gamma_d |X|^T |X| entrywise with d the summation depth, the exact Gram in
    # rational arithmetic; the row-order Gram needs gamma_m
    rng = np.random.default_rng(m + n)
    X = rng.standard_normal((m, n)) * np.exp(rng.uniform(-3, 3, size=(m, 1)))
    A = oracle.gram_chunked(X, chunk)
    d = oracle.gram_depth(m, chunk)
    g = d * U / (1 - d * U)
    absg = np.abs(X).T @ np.abs(X)
    Xf = [[Fraction(v) for v in row] for row in X]
    for i in range(n):
        for j in range(i, n):
            exact = sum(r[i] * r[j] for r in Xf)
            err = abs(Fraction(A[i, j]) - exact)
            assert err <= Fraction(g * absg[i, j] * (1 + 1e-12)), (i, j)


def test_depth_shift_reduces_to_the_paper_shift():
    for m, n in ((1000, 30), (100, 100), (1 << 22, 64)):
        for nrm in (1.0, 0.37, 2.5e3):
            assert oracle.shift_depth(m, n, nrm) == oracle.shift(m, n, nrm)
    # smaller depth, proportionally smaller mn term
    a1 = oracle.shift_depth(1000, 50, 1.0) - oracle.shift_depth(0, 50, 1.0)
    a2 = oracle.shift_depth(250, 50, 1.0) - oracle.shift_depth(0, 50, 1.0)
    assert abs(a1 / a2 - 4.0) < 1e-12


@pytest.mark.parametrize("m,n,kappa,chunk", [(1 << 16, 32, 1e15, 256), (20000, 64, 1e14, 128),
                                             (5000, 17, 1e12, 64)])
def test_depth_mode_kappa_reduction_and_fewer_passes(m, n, kappa, chunk):
    # the first factor's kappa follows the exact-arithmetic form sqrt(sigma_n^2 + s) /
    # (sigma_n sqrt(1 + s)) (Section 4.1) with the depth shift; the smaller shift never needs more
    # passes than the paper's, and the result meets the invariants
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(1, 700 + n))
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, shift_mode=oracle.SHIFT_DEPTH, gram_chunk=chunk,
                    history=True)
    rp = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert r.status == oracle.OK and rp.status == oracle.OK
    assert r.passes <= rp.passes
    d = oracle.gram_depth(m, chunk)
    sv = np.linalg.svd(X, compute_uv=False)
    s = oracle.shift_depth(d, n, sv[0] ** 2)
    assert abs(r.shifts[0] / s - 1) < 1e-9
    np.testing.assert_array_equal(r.grams[0], oracle.gram_chunked(X, chunk))
    exact = (sv[0] / np.sqrt(sv[0] ** 2 + s)) / (sv[-1] / np.sqrt(sv[-1] ** 2 + s))
    k1 = accuracy.cond2(oracle.trsm_rows(X, r.rts[0]))
    assert abs(k1 / exact - 1) < 0.10
    om, _ = accuracy.orthogonality(r.Q)
    assert om <= 1e-13 and accuracy.residual(X, r.Q, r.R) <= 1e-13


def test_depth_mode_invalid_combinations():
    X = synth.randsvd(500, 8, 1e3, seed=5)
    d, o = synth.tridiag_b(500, seed=6)
    assert oracle.scqr(X, shift_mode=oracle.SHIFT_DEPTH, gram_chunk=0).status == oracle.INVALID
    assert oracle.scqr(X, shift_mode=oracle.SHIFT_DEPTH, gram_chunk=64,
                       tridiag=(d, o)).status == oracle.INVALID
