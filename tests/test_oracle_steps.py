"""Pins of the oracle's individual steps against exact arithmetic, closed forms and library
routines (CPU only).  Integer-valued inputs make every binary64 operation exact, so a dropped
term, a wrong index, sign or transposition changes the result bit for bit."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
U = 2.0 ** -53


def int_matrix(rng, m, n, lo=-7, hi=8):
    return rng.integers(lo, hi, size=(m, n)).astype(np.float64)


def exact_gram(X):
    Xi = [[int(v) for v in row] for row in X]
    m, n = len(Xi), len(Xi[0])
    return np.array([[sum(Xi[k][i] * Xi[k][j] for k in range(m)) for j in range(n)]
                     for i in range(n)], dtype=np.float64)


# ---------------------------------------------------------------- Gram (eq:gram)
@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (50, 9), (131, 17)])
def test_gram_exact_on_integers(m, n):
    rng = np.random.default_rng(m * 100 + n)
    X = int_matrix(rng, m, n)
    np.testing.assert_array_equal(oracle.gram(X), exact_gram(X))


def test_gram_orthogonal_columns_closed_form():
    X = np.zeros((6, 3))
    X[0, 0], X[1, 0] = 3.0, 4.0
    X[2, 1] = 2.0
    X[3, 2], X[4, 2], X[5, 2] = 1.0, 2.0, 2.0
    np.testing.assert_array_equal(oracle.gram(X), np.diag([25.0, 4.0, 9.0]))


def test_gram_within_gamma_m_bound_vs_numpy():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5000, 12))
    A = oracle.gram(X)
    gm = 5000 * U / (1 - 5000 * U)
    bound = 2 * gm * (np.abs(X).T @ np.abs(X))  # both sides carry at most gamma_m error
    assert np.all(np.abs(A - X.T @ X) <= bound)
    np.testing.assert_array_equal(A, A.T)


def test_gram_is_row_order_recursive_sum():
    # 1 + 4 * 2^-54 summed left to right stays 1 (each addend is below half an ulp of 1);
    # summing the small terms first, or in reverse order, gives 1 + 2^-52.
    X = np.array([[1.0]] + [[2.0 ** -27]] * 4)
    assert oracle.gram(X)[0, 0] == 1.0
    assert oracle.gram(X[::-1].copy())[0, 0] == 1.0 + 2.0 ** -52


def test_gram_thread_count_invariant():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3000, 13))
    t = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        A1 = oracle.gram(X)
        oracle.set_num_threads(3)
        A3 = oracle.gram(X)
    finally:
        oracle.set_num_threads(t)
    np.testing.assert_array_equal(A1, A3)


def dense_tridiag(d, o):
    B = np.diag(d)
    if o.size:
        B += np.diag(o, 1) + np.diag(o, -1)
    return B


@pytest.mark.parametrize("m,n", [(1, 1), (2, 2), (9, 4), (64, 7)])
def test_gram_tridiag_exact_on_integers(m, n):
    rng = np.random.default_rng(m + 7 * n)
    X = int_matrix(rng, m, n)
    d = rng.integers(1, 9, size=m).astype(np.float64)
    o = rng.integers(-3, 4, size=m - 1).astype(np.float64)
    B = dense_tridiag(d, o)
    Bi = [[int(v) for v in row] for row in B]
    Xi = [[int(v) for v in row] for row in X]
    exact = np.array([[sum(Xi[k][i] * Bi[k][l] * Xi[l][j] for k in range(m) for l in range(m))
                       for j in range(n)] for i in range(n)], dtype=np.float64)
    np.testing.assert_array_equal(oracle.gram_tridiag(X, d, o), exact)
    np.testing.assert_array_equal(oracle.gram_dense(X, B), exact)


def test_gram_tridiag_identity_equals_euclidean_bitwise():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((400, 11))
    np.testing.assert_array_equal(oracle.gram_tridiag(X, np.ones(400), np.zeros(399)),
                                  oracle.gram(X))


def test_gram_f32_error_bound_and_exact_small_integers():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2000, 10))
    for chain in (1, 16, 64):
        A = oracle.gram_f32(X, chain)
        bound = (chain + 3) * oracle.U32 * (np.abs(X).T @ np.abs(X)) * 1.01
        assert np.all(np.abs(A - X.T @ X) <= bound)
    Xi = int_matrix(rng, 300, 6)  # products and chain sums stay exact in binary32
    np.testing.assert_array_equal(oracle.gram_f32(Xi, 64), exact_gram(Xi))


# ---------------------------------------------------------------- eigenvalues (norm estimate)
def test_sym_eig_closed_form_and_vs_lapack():
    np.testing.assert_allclose(oracle.sym_eig(np.array([[2.0, 1.0], [1.0, 2.0]])), [1.0, 3.0],
                               rtol=0, atol=1e-15)
    rng = np.random.default_rng(4)
    for n in (1, 5, 40):
        W, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.sort(rng.uniform(-3, 5, size=n))
        A = (W * lam) @ W.T
        A = 0.5 * (A + A.T)
        np.testing.assert_allclose(oracle.sym_eig(A), lam, rtol=0, atol=1e-13)
        assert abs(oracle.lambda_max(A) - np.linalg.eigvalsh(A)[-1]) <= 1e-13


# ---------------------------------------------------------------- Cholesky (Algorithm 1 line 3)
def int_upper(rng, n, diag_pow2=False):
    R = np.triu(rng.integers(-5, 6, size=(n, n)).astype(np.float64), 1)
    if diag_pow2:
        np.fill_diagonal(R, 2.0 ** rng.integers(0, 3, size=n))
    else:
        np.fill_diagonal(R, rng.integers(1, 6, size=n))
    return R


@pytest.mark.parametrize("n", [1, 2, 6, 15])
def test_chol_exact_on_integer_factor(n):
    rng = np.random.default_rng(n)
    R0 = int_upper(rng, n, diag_pow2=True)
    A = R0.T @ R0  # exact integers
    R, info = oracle.chol_upper(A)
    assert info == 0
    np.testing.assert_array_equal(R, R0)
    # the shift enters on the diagonal only: chol(A - sI + sI) == R0
    s = 4.0
    R2, info2 = oracle.chol_upper(A - s * np.eye(n), s)
    assert info2 == 0
    np.testing.assert_array_equal(R2, R0)


def test_chol_vs_lapack_and_backward_error():
    rng = np.random.default_rng(9)
    Xm = rng.standard_normal((200, 30))
    A = Xm.T @ Xm
    R, info = oracle.chol_upper(A, 0.5)
    assert info == 0
    L = np.linalg.cholesky(A + 0.5 * np.eye(30))
    np.testing.assert_allclose(R, L.T, rtol=1e-12, atol=1e-12)
    # R^T R = A + sI + E2 with |E2| <= gamma_{n+1} |R^T||R| (Section 3.1.2)
    g = 31 * U / (1 - 31 * U)
    assert np.all(np.abs(R.T @ R - (A + 0.5 * np.eye(30))) <= 2 * g * (np.abs(R.T) @ np.abs(R)))


def test_chol_breakdown_reporting():
    R, info = oracle.chol_upper(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert info == 2
    R, info = oracle.chol_upper(np.array([[0.0, 0.0], [0.0, 1.0]]))
    assert info == 1
    R, info = oracle.chol_upper(np.array([[1.0, np.nan], [np.nan, 1.0]]))
    assert info == 2
    R, info = oracle.chol_upper(np.array([[-1.0]]), 2.0)  # shift rescues the pivot
    assert info == 0 and R[0, 0] == 1.0


# ---------------------------------------------------------------- TRSM (Algorithm 1 line 4)
@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (77, 12)])
def test_trsm_exact_on_integer_factors(m, n):
    rng = np.random.default_rng(m + n)
    R0 = int_upper(rng, n, diag_pow2=True)
    Q0 = int_matrix(rng, m, n, -3, 4)
    X = Q0 @ R0
    np.testing.assert_array_equal(oracle.trsm_rows(X, R0), Q0)


def test_trsm_rowwise_backward_stable_vs_scipy():
    rng = np.random.default_rng(11)
    n = 24
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    X = rng.standard_normal((500, n))
    Q = oracle.trsm_rows(X, R)
    ref = scipy.linalg.solve_triangular(R, X.T, trans="T", lower=False).T
    np.testing.assert_allclose(Q, ref, rtol=1e-11, atol=1e-12)
    # row-wise residual |q_i^T R - x_i^T| <= gamma_n |q_i^T| |R| (backward error per row)
    g = n * U / (1 - n * U)
    assert np.all(np.abs(Q @ R - X) <= 2 * g * (np.abs(Q) @ np.abs(R)) + 1e-300)


def test_trmm_exact_on_integers():
    rng = np.random.default_rng(12)
    A = int_upper(rng, 9)
    B = int_upper(rng, 9)
    np.testing.assert_array_equal(oracle.trmm_upper(A, B), A @ B)


def test_gershgorin_tridiag():
    d = np.array([2.5, 3.0, 10.0, 2.0])
    o = np.array([-1.0, -1.0, 0.5])
    assert oracle.gershgorin_tridiag(d, o) == 11.5
    B = dense_tridiag(d, o)
    assert oracle.gershgorin_tridiag(d, o) >= np.linalg.eigvalsh(B)[-1]


# ---------------------------------------------------------------- shift (eq:finds2, eq:finds2B)
def test_unit_roundoff_matches_paper():
    assert oracle.U == GOLD["unit_roundoff"]["u"] == 2.0 ** -53


@pytest.mark.parametrize("tab", ["table1", "table2"])
def test_shift_formula_reproduces_printed_kappa_reduction(tab):
    t = GOLD[tab]
    m, n, kappa = t["m"], t["n"], t["kappa"]
    alpha = oracle.shift(m, n, 1.0)  # ||X||_2 = 1 for randsvd inputs
    predicted = np.sqrt(alpha) * kappa  # kappa(Q^(1)) ~ sqrt(alpha) kappa(X) (eq:redcond)
    assert abs(predicted / t["kappa_q"][0] - 1) < 0.005
    # the printed sqrt(alpha) column is not the paper's own formula (documented reading)
    assert abs(np.sqrt(alpha) / t["sqrt_alpha_printed"] - 1) > 0.5


def test_shift_formula_table2_needs_the_n_squared_term():
    t = GOLD["table2"]
    m, n = t["m"], t["n"]
    without = np.sqrt(11 * m * n * U) * t["kappa"]
    assert abs(without / t["kappa_q"][0] - 1) > 0.2  # the full formula is the one printed


def test_shift_oblique_reproduces_table3_factor():
    t = GOLD["table3"]
    alpha = oracle.shift(t["m"], t["n"], 1.0, 1.0, oblique=True)
    assert abs(np.sqrt(alpha * t["kappa_b"]) / t["sqrt_alpha_kappa_b"] - 1) < 0.005


def test_shift_remark_value():
    r = GOLD["remark_shift"]
    s = oracle.shift(r["m"], r["n"], 1.0)
    assert abs(s - 6.418e-11) < 1e-13  # full formula
    # the printed 6.1e-11 equals 11 m n u, i.e. the n(n+1) term dropped (documented reading)
    assert abs(11 * r["m"] * r["n"] * U / r["s_printed"] - 1) < 0.01


def test_shift_modes_scale():
    assert oracle.shift(100, 10, 4.0, mode=oracle.SHIFT_SMALL) == U * 4.0
    assert oracle.shift(100, 10, 4.0, 2.0, oblique=True, mode=oracle.SHIFT_SMALL) == U * 8.0
    assert oracle.shift(100, 10, 4.0, mode=oracle.SHIFT_CUSTOM, alpha=1e-3) == 4e-3
    assert oracle.shift(1000, 10, 2.0) == 11 * (1000 * 10 + 10 * 11) * U * 2.0
    s = oracle.shift(1000, 10, 2.0, 3.0, oblique=True)
    assert abs(s - 11 * (2 * 1000 * np.sqrt(1000 * 10) + 110) * U * 6.0) <= 1e-12 * s
    s32 = oracle.shift_f32(10, 64, 2.0)
    assert abs(s32 - 11 * (66 * 10 * oracle.U32 + 110 * U) * 2.0) <= 1e-15 * s32
