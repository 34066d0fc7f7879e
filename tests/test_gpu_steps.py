"""GPU parity of the individual steps against the oracle, through the C ABI.

Integer-valued inputs keep every binary64 (and binary32) operation exact, so the GPU Gram,
oblique Gram and substitution must equal the oracle bit for bit whatever their summation
order; random inputs are checked against the oracle within the rounding bounds of Section 3.
Shapes span several 16-column tiles and 64-row panels with ragged tails."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
U = 2.0 ** -53

SHAPES = [(1, 1), (16, 16), (17, 5), (100, 16), (1000, 17), (4097, 32), (70001, 33), (5000, 64),
          (3000, 65), (20000, 100), (10000, 128), (4000, 129), (3000, 200), (2000, 256)]


@pytest.fixture(scope="module")
def scqr():
    import paper_1809_11085_amd as s
    assert torch.cuda.is_available()
    s.lib()
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,n", SHAPES)
def test_gram_bit_exact_on_integers(scqr, m, n):
    rng = np.random.default_rng(m * 7 + n)
    X = rng.integers(-7, 8, size=(m, n)).astype(np.float64)
    G = host(scqr.gram(dev(X)))
    exact = (X.astype(np.int64).T @ X.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(G, exact)
    np.testing.assert_array_equal(G, oracle.gram(X))


@pytest.mark.parametrize("m,n", [(1000, 17), (70001, 64), (20000, 128), (3000, 256)])
def test_gram_random_within_bound(scqr, m, n):
    X = synth.randsvd(m, n, 1e8, seed=m + n)
    G = host(scqr.gram(dev(X)))
    Go = oracle.gram(X)
    bound = 2 * (m * U / (1 - m * U)) * (np.abs(X).T @ np.abs(X))
    assert np.all(np.abs(G - Go) <= bound)
    np.testing.assert_array_equal(G, G.T)


def test_gram_strided_input(scqr):
    rng = np.random.default_rng(3)
    big = rng.integers(-5, 6, size=(5000, 80)).astype(np.float64)
    Xt = dev(big)[:, 3:43]  # ld = 80, n = 40
    G = host(scqr.gram(Xt))
    X = big[:, 3:43]
    np.testing.assert_array_equal(G, (X.astype(np.int64).T @ X.astype(np.int64)).astype(np.float64))


@pytest.mark.parametrize("m,n", [(2, 1), (65, 16), (1000, 17), (20001, 64), (5000, 128), (3000, 256)])
def test_oblique_gram_bit_exact_on_integers(scqr, m, n):
    rng = np.random.default_rng(m + 3 * n)
    X = rng.integers(-5, 6, size=(m, n)).astype(np.float64)
    d = rng.integers(1, 9, size=m).astype(np.float64)
    o = rng.integers(-3, 4, size=m - 1).astype(np.float64)
    G = host(scqr.gram(dev(X), B=(dev(d), dev(o))))
    Xi = X.astype(np.int64)
    BX = d.astype(np.int64)[:, None] * Xi
    BX[:-1] += o.astype(np.int64)[:, None] * Xi[1:]
    BX[1:] += o.astype(np.int64)[:, None] * Xi[:-1]
    exact = (Xi.T @ BX).astype(np.float64)
    exact = np.triu(exact) + np.triu(exact, 1).T
    np.testing.assert_array_equal(G, exact)
    np.testing.assert_array_equal(G, oracle.gram_tridiag(X, d, o))


def int_upper(rng, n):
    R = np.triu(rng.integers(-4, 5, size=(n, n)).astype(np.float64), 1)
    np.fill_diagonal(R, 2.0 ** rng.integers(0, 3, size=n))
    return R


@pytest.mark.parametrize("m,n", [(1, 1), (17, 5), (1000, 16), (4097, 33), (3000, 64), (2000, 65),
                                 (1500, 128), (700, 200), (500, 256)])
def test_trsm_bit_exact_on_integer_factors(scqr, m, n):
    rng = np.random.default_rng(m + n)
    R0 = int_upper(rng, n)
    Q0 = rng.integers(-2, 3, size=(m, n)).astype(np.float64)
    X = Q0 @ R0
    assert np.max(np.abs(X)) < 2 ** 40
    Q = host(scqr.trsm(dev(X), dev(R0)))
    np.testing.assert_array_equal(Q, Q0)
    np.testing.assert_array_equal(Q, oracle.trsm_rows(X, R0))


@pytest.mark.parametrize("m,n", [(5000, 30), (20000, 64), (4000, 128), (1000, 256)])
def test_trsm_random_rowwise_backward_stable(scqr, m, n):
    rng = np.random.default_rng(n)
    R = np.triu(rng.standard_normal((n, n))) + np.diag(3 + rng.random(n))
    X = rng.standard_normal((m, n))
    Q = host(scqr.trsm(dev(X), dev(R)))
    g = (n + 1) * U / (1 - (n + 1) * U)
    assert np.all(np.abs(Q @ R - X) <= 3 * g * (np.abs(Q) @ np.abs(R)) + 1e-300)
    Qo = oracle.trsm_rows(X, R)
    assert np.max(np.abs(Q - Qo)) <= 1e-10 * np.max(np.abs(Qo))


def test_trsm_in_place(scqr):
    rng = np.random.default_rng(9)
    n = 48
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    X = rng.standard_normal((9000, n))
    Xt = dev(X)
    Q = scqr.trsm(Xt, dev(R), out=Xt)
    assert Q.data_ptr() == Xt.data_ptr()
    Qo = oracle.trsm_rows(X, R)
    assert np.max(np.abs(host(Q) - Qo)) <= 1e-12 * np.max(np.abs(Qo))
