"""GPU parity of the oblique factorization with a general sparse SPD B in compressed sparse rows
(Section 7; Algorithms 4 and 5) against the oracle, through the C ABI.

* The B-Gram X^T B X (Y = B X formed row by row, summed in storage order): bit for bit on
  integer inputs, where every order gives the exact result; on random inputs within
  2 gamma_{m + r} |X|^T |B| |X| of the oracle's (both within gamma_{m + r} of the exact Gram,
  r the largest number of entries in a row).
* The first shift follows equation (eq:finds2B) with ||X||_2 from the power iteration and the
  Gershgorin bound of B, which equals the oracle's bit for bit (both sum each row's absolute
  values in storage order).
* Passes 2 and later: every traced B-Gram is checked against the oracle's B-Gram of the
  replayed iterate.
* Invariants: ||Q^T B Q - I||_2 <= 1e-13 (compensated), ||X - QR||_F / ||X||_F <= 1e-13; the pass
  count of the oracle for kappa <= 1e10; factors equal to the oracle's for kappa <= 1e6.
* Index errors in the caller's CSR arrays are caught by the kernel's own checks (no access
  outside the arrays) and reported as SCQR_E_INVALID.
"""
import numpy as np
import pytest
import torch

import accuracy
import oracle
import synth

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def scqr():
    import paper_1809_11085_amd as s
    assert torch.cuda.is_available()
    s.lib()
    return s


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dev_csr(scqr, B):
    return scqr.CsrB(torch.from_numpy(B.row_ptr).cuda(), torch.from_numpy(B.col).cuda(),
                     torch.from_numpy(B.val).cuda())


def make_b(kind, m, seed):
    if kind == "rand":
        return synth.random_pattern_b(m, 48, 512, seed=seed)
    return synth.stencil_b(m, kind, seed=seed)


def csr_tuple(B):
    return (B.row_ptr, B.col, B.val)


@pytest.mark.parametrize("n", [1, 7, 16, 33, 64, 100, 128, 200, 256])
def test_csr_gram_exact_on_integers(scqr, n):
    m = 1500 + n
    rng = np.random.default_rng(n)
    X = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
    B = synth.stencil_b(m, "27pt", seed=n)
    Bi = synth.CsrB(B.row_ptr, B.col, np.rint(B.val * 2.0))  # integer, symmetric, same pattern
    G = host(scqr.gram(torch.from_numpy(X).cuda(), B=dev_csr(scqr, Bi)))
    np.testing.assert_array_equal(G, oracle.gram_csr(X, csr_tuple(Bi)))


@pytest.mark.parametrize("kind,m,n", [("5pt", 40000, 64), ("27pt", 30011, 32), ("rand", 20000, 128),
                                      ("27pt", 5000, 256), ("rand", 3000, 16)])
def test_csr_gram_random_within_bound(scqr, kind, m, n):
    X = synth.randsvd(m, n, 1e6, seed=synth.seed_for(5, m + n))
    B = make_b(kind, m, seed=m)
    G = host(scqr.gram(torch.from_numpy(X).cuda(), B=dev_csr(scqr, B)))
    Go = oracle.gram_csr(X, csr_tuple(B))
    r = int(np.diff(B.row_ptr).max())
    g = (m + r) * U / (1 - (m + r) * U)
    absb = oracle.gram_csr(np.abs(X), (B.row_ptr, B.col, np.abs(B.val)))
    assert np.all(np.abs(G - Go) <= 2 * g * absb + 1e-300)
    np.testing.assert_array_equal(G, G.T)


@pytest.mark.parametrize("kind,m,n,kappa", [("5pt", 40000, 32, 1e10), ("27pt", 20000, 64, 1e6),
                                            ("rand", 20000, 16, 1e12), ("27pt", 30000, 128, 1e8),
                                            ("5pt", 4000, 256, 1e5), ("rand", 6001, 100, 1e4),
                                            ("5pt", 1000, 1, 1.0)])
def test_csr_qr_against_oracle(scqr, kind, m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(5, 3 * m + n))
    B = make_b(kind, m, seed=m + 1)
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), B=dev_csr(scqr, B), schedule="adaptive", trace=True)
    assert info.status == scqr.OK, info
    Qh, Rh = host(Q), host(R)
    assert accuracy.orthogonality(Qh, csr=csr_tuple(B))[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
    assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)
    bn = oracle.gershgorin_csr(csr_tuple(B))
    assert info.bnorm == bn
    lam = oracle.lambda_max(oracle.gram(X))
    s_exact = oracle.shift(m, n, lam, bnorm=bn, oblique=True)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-12)
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, csr=csr_tuple(B))
    assert ro.status == oracle.OK
    if kappa <= 1e10:
        assert ro.passes == info.passes
    if kappa <= 1e6:
        assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)
        assert np.max(np.abs(Qh - ro.Q)) <= 1e-10
    # replay: the B-Gram of every later pass against the oracle's B-Gram of the same iterate
    tr = info.trace.cpu().numpy()
    r = int(np.diff(B.row_ptr).max())
    g = (m + r) * U / (1 - (m + r) * U)
    absv = (B.row_ptr, B.col, np.abs(B.val))
    Qd = torch.from_numpy(X).cuda()
    for p in range(info.passes):
        if p >= 1:
            Qp = host(Qd)
            Go = oracle.gram_csr(Qp, csr_tuple(B))
            assert np.all(np.abs(tr[p, 0] - Go) <= 2 * g * oracle.gram_csr(np.abs(Qp), absv) + 1e-300), p
        Qd = scqr.trsm(Qd, torch.from_numpy(np.ascontiguousarray(tr[p, 1])).cuda())
    np.testing.assert_array_equal(host(Qd), Qh)


def test_csr_of_tridiagonal_matches_tridiagonal_path(scqr):
    m, n = 50000, 48
    X = synth.randsvd(m, n, 1e6, seed=synth.seed_for(5, 77))
    d, o = synth.tridiag_b(m, seed=synth.seed_for(5, 78))
    rows = np.concatenate([np.arange(1, m), np.arange(m), np.arange(m - 1)])
    cols = np.concatenate([np.arange(m - 1), np.arange(m), np.arange(1, m)])
    vals = np.concatenate([o, d, o])
    order = np.lexsort((cols, rows))
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    B = synth.CsrB(rp, cols[order].astype(np.int32), vals[order])
    Xd = torch.from_numpy(X).cuda()
    Qc, Rc, ic = scqr.qr(Xd, B=dev_csr(scqr, B))
    Qt, Rt, it = scqr.qr(Xd, B=(torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda()))
    assert ic.status == it.status == scqr.OK and ic.passes == it.passes
    assert ic.bnorm == it.bnorm
    assert torch.linalg.norm(Rc - Rt) <= 1e-11 * torch.linalg.norm(Rt)
    assert torch.max(torch.abs(Qc - Qt)) <= 1e-11


def test_csr_user_bnorm_and_in_place(scqr):
    m, n = 12000, 24
    X = synth.randsvd(m, n, 1e9, seed=synth.seed_for(5, 90))
    B = make_b("27pt", m, seed=91)
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), B=dev_csr(scqr, B), bnorm=500.0)
    assert info.status == scqr.OK and info.bnorm == 500.0
    Xd = torch.from_numpy(X).cuda()
    Q2, R2, _ = scqr.qr(Xd, B=dev_csr(scqr, B), bnorm=500.0, inplace=True)
    assert Q2.data_ptr() == Xd.data_ptr() and torch.equal(Q2, Q) and torch.equal(R2, R)


def test_csr_index_errors_reported(scqr):
    # every bad index below is caught by the kernel's own range checks before it is used
    m, n = 3000, 8
    X = torch.from_numpy(synth.randsvd(m, n, 1e3, seed=5)).cuda()
    B = make_b("5pt", m, seed=6)
    col = B.col.copy()
    col[17] = m  # a column past the last row
    _, _, info = scqr.qr(X, B=scqr.CsrB(torch.from_numpy(B.row_ptr).cuda(), torch.from_numpy(col).cuda(),
                                        torch.from_numpy(B.val).cuda()), check="status")
    assert info.status == scqr.E_INVALID and info.passes == 0
    col[17] = -3
    _, _, info = scqr.qr(X, B=scqr.CsrB(torch.from_numpy(B.row_ptr).cuda(), torch.from_numpy(col).cuda(),
                                        torch.from_numpy(B.val).cuda()), check="status")
    assert info.status == scqr.E_INVALID
    rp = B.row_ptr.copy()
    rp[100] = rp[101] + 1  # decreasing row pointers
    _, _, info = scqr.qr(X, B=scqr.CsrB(torch.from_numpy(rp).cuda(), torch.from_numpy(B.col).cuda(),
                                        torch.from_numpy(B.val).cuda()), check="status")
    assert info.status == scqr.E_INVALID
    # a valid B afterwards, with the same workspace size: unaffected
    _, _, info = scqr.qr(X, B=dev_csr(scqr, B))
    assert info.status == scqr.OK
