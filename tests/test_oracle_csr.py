"""Pins of the oracle's oblique Gram and driver for a general sparse SPD B in compressed sparse
row form (Section 7, oblique inner product; Algorithms 4 and 5 with B stored as CSR).

* Exactness: with integer X and B every product and sum is exact, so X^T B X equals the exact
  integer result whatever the order; also after permuting the entries inside each row.
* Reductions to the already pinned forms, bit for bit on random (non-integer) data: the CSR of a
  tridiagonal B (entries of row k stored as k-1, k, k+1) gives the tridiagonal Gram; the CSR of a
  dense B (all columns, ascending) gives the dense-B Gram; the drivers then agree bit for bit.
* Gershgorin bound: the largest absolute row sum, an upper bound of lambda_max(B).
"""
import numpy as np
import pytest

import oracle
import synth


def csr_of_dense(D):
    m = D.shape[0]
    rows, cols = np.nonzero(D)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return rp, cols.astype(np.int32), D[rows, cols].astype(np.float64)


def csr_of_tridiag(d, o):
    m = d.size
    rows, cols, vals = [], [], []
    for k in range(m):
        if k > 0:
            rows.append(k), cols.append(k - 1), vals.append(o[k - 1])
        rows.append(k), cols.append(k), vals.append(d[k])
        if k + 1 < m:
            rows.append(k), cols.append(k + 1), vals.append(o[k])
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(np.array(rows), minlength=m), out=rp[1:])
    return rp, np.array(cols, dtype=np.int32), np.array(vals)


def test_integer_gram_is_exact():
    rng = np.random.default_rng(5)
    m, n = 300, 9
    X = rng.integers(-20, 21, size=(m, n))
    B = synth.stencil_b(m, "27pt", seed=3)
    Bi = np.rint(B.dense() * 4).astype(np.int64)  # integer symmetric, same pattern
    Bi = np.triu(Bi) + np.triu(Bi, 1).T
    csr = csr_of_dense(Bi.astype(float))
    exact = X.astype(object).T @ (Bi.astype(object) @ X.astype(object))
    A = oracle.gram_csr(X.astype(float), csr)
    np.testing.assert_array_equal(A, np.array(exact, dtype=float))
    # the order of the entries inside a row changes nothing on exact data
    rp, col, val = csr
    perm = np.concatenate([rng.permutation(np.arange(rp[k], rp[k + 1])) for k in range(m)])
    np.testing.assert_array_equal(oracle.gram_csr(X.astype(float), (rp, col[perm], val[perm])), A)


def test_tridiagonal_as_csr_bitwise():
    m, n = 2000, 13
    X = synth.randsvd(m, n, 1e8, seed=7)
    d, o = synth.tridiag_b(m, seed=8)
    csr = csr_of_tridiag(d, o)
    np.testing.assert_array_equal(oracle.gram_csr(X, csr), oracle.gram_tridiag(X, d, o))
    assert oracle.gershgorin_csr(csr) == oracle.gershgorin_tridiag(d, o)


def test_dense_as_csr_bitwise():
    m, n = 150, 7
    X = synth.randsvd(m, n, 1e6, seed=9)
    Bd = synth.dense_spd_b(m, 1e4, seed=10)
    np.testing.assert_array_equal(oracle.gram_csr(X, csr_of_dense(Bd)), oracle.gram_dense(X, Bd))


@pytest.mark.parametrize("kind", ["5pt", "27pt", "rand"])
def test_gershgorin_csr_bounds_lambda_max(kind):
    m = 500
    B = synth.random_pattern_b(m, 48, 60, seed=11) if kind == "rand" else synth.stencil_b(m, kind, seed=11)
    D = B.dense()
    g = oracle.gershgorin_csr((B.row_ptr, B.col, B.val))
    rowsum = np.abs(D).sum(axis=1).max()
    assert abs(g - rowsum) <= 1e-14 * rowsum
    assert g >= np.linalg.eigvalsh(D)[-1]


def test_driver_reduces_to_tridiagonal_and_dense():
    m, n = 3000, 16
    X = synth.randsvd(m, n, 1e12, seed=12)
    d, o = synth.tridiag_b(m, seed=13)
    rt = oracle.scqr(X, schedule=oracle.ADAPTIVE, tridiag=(d, o), history=True)
    rc = oracle.scqr(X, schedule=oracle.ADAPTIVE, csr=csr_of_tridiag(d, o), history=True)
    assert rt.status == rc.status == oracle.OK and rt.passes == rc.passes
    np.testing.assert_array_equal(rc.Q, rt.Q)
    np.testing.assert_array_equal(rc.R, rt.R)
    assert rc.shifts == rt.shifts
    m2 = 200
    X2 = synth.randsvd(m2, 6, 1e9, seed=14)
    Bd = synth.dense_spd_b(m2, 1e3, seed=15)
    r1 = oracle.scqr(X2, schedule=oracle.ADAPTIVE, B=Bd, bnorm=1.5)
    r2 = oracle.scqr(X2, schedule=oracle.ADAPTIVE, csr=csr_of_dense(Bd), bnorm=1.5)
    assert r1.passes == r2.passes
    np.testing.assert_array_equal(r2.Q, r1.Q)
    np.testing.assert_array_equal(r2.R, r1.R)


@pytest.mark.parametrize("kind,n,kappa", [("5pt", 16, 1e12), ("27pt", 24, 1e8), ("rand", 8, 1e15)])
def test_driver_invariants_sparse(kind, n, kappa):
    # Algorithm 5's guarantee: Q^T B Q = I and X = Q R to working accuracy
    m = 4000
    B = synth.random_pattern_b(m, 48, 100, seed=16) if kind == "rand" else synth.stencil_b(m, kind, seed=16)
    X = synth.randsvd(m, n, kappa, seed=17)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, csr=(B.row_ptr, B.col, B.val))
    assert r.status == oracle.OK
    D = B.dense()
    assert np.linalg.norm(r.Q.T @ D @ r.Q - np.eye(n), 2) <= 1e-12
    assert np.linalg.norm(X - r.Q @ r.R) <= 1e-13 * np.linalg.norm(X)
    assert np.all(np.diag(r.R) > 0)
    # first shift: equation (eq:finds2B) with the exact ||X||_2 and the Gershgorin bound
    s = oracle.shift(m, n, np.linalg.norm(X, 2) ** 2, bnorm=oracle.gershgorin_csr((B.row_ptr, B.col, B.val)),
                     oblique=True)
    assert abs(r.shifts[0] / s - 1) <= 1e-12


def test_malformed_csr_rejected():
    X = np.ones((4, 2))
    with pytest.raises(ValueError):
        oracle.gram_csr(X, (np.array([0, 1, 2, 3]), np.array([0, 1, 2]), np.ones(3)))  # short row_ptr
    with pytest.raises(ValueError):
        oracle.gram_csr(X, (np.array([0, 1, 2, 3, 4]), np.array([0, 1, 2, 4]), np.ones(4)))  # column 4
