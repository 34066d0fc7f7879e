"""Pins of the compensated accuracy measurements (CPU): the Dot2 Gram (Ogita, Rump and Oishi's
compensated dot product) and the compensated residual that every orthogonality and residual
bound of the test suite and of the benchmark goes through.  Each construction has an exact
answer known without the module: integer or power-of-two data whose sums are exact, an
orthonormal Hadamard basis, and rational arithmetic for the expected values."""
from fractions import Fraction

import numpy as np
import pytest

import accuracy

U = 2.0 ** -53


def hadamard(m):
    H = np.array([[1.0]])
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


def exact_gram(Q):
    Qf = [[Fraction(float(v)) for v in row] for row in Q]
    n = len(Qf[0])
    return [[sum((r[i] * r[j] for r in Qf), Fraction(0)) for j in range(n)] for i in range(n)]


def test_dot2_exact_where_recursive_summation_rounds():
    # a = (1, 2^-27, 1), b = (1, 2^-27, -1): a^T b = 2^-54 exactly.  Recursive binary64 summation
    # gives (1 + 2^-54) - 1 = 0 (the 2^-54 is lost in the first addition); Dot2 keeps it.
    Q = np.array([[1.0, 1.0], [2.0 ** -27, 2.0 ** -27], [1.0, -1.0]])
    G = accuracy.gram(Q)
    assert G[0, 1] == 2.0 ** -54 and G[1, 0] == 2.0 ** -54
    plain = 0.0
    for k in range(3):
        plain = plain + Q[k, 0] * Q[k, 1]
    assert plain == 0.0
    # diagonal: 2 + 2^-54 rounds to 2 (faithful)
    assert G[0, 0] == 2.0


def test_dot2_gram_exact_on_integers():
    rng = np.random.default_rng(3)
    Q = rng.integers(-1000, 1000, size=(500, 7)).astype(np.float64)
    G = accuracy.gram(Q)
    E = exact_gram(Q)
    for i in range(7):
        for j in range(7):
            assert G[i, j] == float(E[i][j])


@pytest.mark.parametrize("m,n", [(256, 16), (1024, 40), (64, 64)])
def test_orthogonality_of_scaled_orthonormal_columns(m, n):
    # Q = H[:, :n] / sqrt(m) is exactly orthonormal (entries +-2^-k); scaling column j by
    # (1 + d_j), d_j = (j + 1) 2^-30, gives Q^T Q - I = diag((1 + d_j)^2 - 1) exactly, so
    # ||Q^T Q - I||_2 = max_j (2 d_j + d_j^2) and ||.||_F is the root of their squares
    H = hadamard(m)[:, :n] / np.sqrt(m)
    assert accuracy.orthogonality(H) == (0.0, 0.0)
    d = np.array([(j + 1) * 2.0 ** -30 for j in range(n)])
    Q = H * (1.0 + d)
    om2, omf = accuracy.orthogonality(Q)
    ex = [(1 + Fraction(float(dj))) ** 2 - 1 for dj in d]
    ex2 = float(max(ex))
    exf = float(sum(e * e for e in ex)) ** 0.5
    assert abs(om2 - ex2) <= 8 * U and abs(omf - exf) <= 8 * U * np.sqrt(n)
    # the off-diagonal part is zero to double-double accuracy
    G = accuracy.gram(Q)
    assert np.max(np.abs(G - np.diag(np.diag(G)))) <= 1e-30


def test_residual_with_known_perturbation():
    # X = Q R + E with integer Q, R (Q R exact) and E of power-of-two entries at known places:
    # ||X - Q R||_F / ||X||_F is known exactly in rational arithmetic
    rng = np.random.default_rng(4)
    m, n = 300, 9
    Q = rng.integers(-20, 21, size=(m, n)).astype(np.float64)
    R = np.triu(rng.integers(-20, 21, size=(n, n))).astype(np.float64)
    R[np.diag_indices(n)] = np.abs(R[np.diag_indices(n)]) + 1
    X = Q @ R
    E = np.zeros_like(X)
    for (i, j, e) in [(3, 2, 2.0 ** -20), (77, 0, -2.0 ** -18), (299, 8, 2.0 ** -25), (150, 4, 2.0 ** -19)]:
        E[i, j] = e
    X = X + E
    assert np.array_equal(X - Q @ R, E)   # every entry is exact
    Xf = sum(Fraction(float(v)) ** 2 for v in X.ravel())
    Ef = sum(Fraction(float(v)) ** 2 for v in E.ravel())
    want = (float(Ef) / float(Xf)) ** 0.5
    got = accuracy.residual(X, Q, R)
    assert abs(got / want - 1) <= 1e-14
    # only the upper triangle of R is read
    Rl = R + np.tril(np.ones((n, n)), -1) * 1e6
    assert accuracy.residual(X, Q, Rl) == got
    rows = np.arange(m)
    assert abs(accuracy.residual_rows(X, Q, R, rows) / want - 1) <= 1e-14
    assert accuracy.residual(Q @ R, Q, R) == 0.0


def test_tridiagonal_dot2_gram_exact_on_integers():
    rng = np.random.default_rng(5)
    m, n = 200, 6
    Q = rng.integers(-50, 51, size=(m, n)).astype(np.float64)
    diag = rng.integers(3, 9, size=m).astype(np.float64)
    off = -rng.integers(0, 3, size=m - 1).astype(np.float64)
    G = accuracy.gram(Q, (diag, off))
    Bm = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    Qi = Q.astype(np.int64)
    Bi = Bm.astype(np.int64)
    want = Qi.T @ (Bi @ Qi)   # exact in int64
    assert np.array_equal(G, want.astype(np.float64))
    # B = I reduces to the Euclidean Gram
    Gi = accuracy.gram(Q, (np.ones(m), np.zeros(m - 1)))
    assert np.array_equal(Gi, accuracy.gram(Q))


def test_tridiagonal_dot2_keeps_cancelled_low_part():
    # rows (1, 1), (2^-27, 2^-27), (1, -1) with B = diag(1, 1, 1): the (0, 1) entry is 2^-54 as in
    # the Euclidean case; with B = diag(1, 4, 1) it is 4 * 2^-54 = 2^-52
    Q = np.array([[1.0, 1.0], [2.0 ** -27, 2.0 ** -27], [1.0, -1.0]])
    assert accuracy.gram(Q, (np.ones(3), np.zeros(2)))[0, 1] == 2.0 ** -54
    assert accuracy.gram(Q, (np.array([1.0, 4.0, 1.0]), np.zeros(2)))[0, 1] == 2.0 ** -52


def _csr_of_dense(D):
    m = D.shape[0]
    rows, cols = np.nonzero(D)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return rp, cols.astype(np.int32), D[rows, cols]


def test_csr_dot2_gram_exact_on_integers_and_cancellation():
    rng = np.random.default_rng(6)
    m, n = 150, 5
    Q = rng.integers(-40, 41, size=(m, n)).astype(np.float64)
    Bi = rng.integers(-3, 4, size=(m, m)) * (rng.random((m, m)) < 0.05)
    Bi = np.triu(Bi, 1) + np.triu(Bi, 1).T + np.diag(rng.integers(5, 9, size=m))
    G = accuracy.gram(Q, csr=_csr_of_dense(Bi.astype(np.float64)))
    want = Q.astype(np.int64).T @ (Bi @ Q.astype(np.int64))
    assert np.array_equal(G, want.astype(np.float64))
    # the cancellation of the tridiagonal pin, through CSR: B = diag(1, 4, 1)
    Q3 = np.array([[1.0, 1.0], [2.0 ** -27, 2.0 ** -27], [1.0, -1.0]])
    assert accuracy.gram(Q3, csr=_csr_of_dense(np.diag([1.0, 4.0, 1.0])))[0, 1] == 2.0 ** -52


def test_csr_dot2_gram_matches_tridiagonal():
    rng = np.random.default_rng(7)
    m, n = 500, 4
    Q = rng.standard_normal((m, n))
    d = 2.0 + rng.random(m)
    o = -rng.random(m - 1)
    Bm = np.diag(d) + np.diag(o, 1) + np.diag(o, -1)
    Gc = accuracy.gram(Q, csr=_csr_of_dense(Bm))
    Gt = accuracy.gram(Q, (d, o))
    # both compensated sums are accurate to about u^2 relative to |Q|^T |B| |Q|: equal up to
    # the final rounding
    scale = np.abs(Q).T @ np.abs(Bm) @ np.abs(Q)
    assert np.all(np.abs(Gc - Gt) <= 2.0 ** -52 * scale)
