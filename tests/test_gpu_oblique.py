"""GPU parity of the oblique factorization (Algorithms 4 and 5) with a tridiagonal SPD B against
the oracle, through the C ABI.

* The first pass uses the oblique shift of equation (eq:finds2B),
  s = 11(2m sqrt(mn) + n(n+1)) u ||X||_2^2 ||B||_2, with ||X||_2 the Euclidean norm (power
  iteration on X^T X) and ||B||_2 bounded by the Gershgorin maximum of B's rows; both are
  compared with the oracle's values on the same input.
* Later passes are B-orthogonal Cholesky QR steps on Q^T B Q (the reading of Algorithm 5 whose
  B = I case is Algorithm 3).
* Invariants: ||Q^T B Q - I||_2 <= 1e-13 (compensated Gram), ||X - QR||_F / ||X||_F <= 1e-13,
  positive diagonal; factors equal to the oracle's for kappa <= 1e6; the pass count of the
  oracle for kappa <= 1e10.
"""
import numpy as np
import pytest
import torch

import accuracy
import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scqr():
    import paper_1809_11085_amd as s
    assert torch.cuda.is_available()
    s.lib()
    return s


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,n,kappa", [(20000, 32, 1e10), (5000, 64, 1e6), (4099, 17, 1e12),
                                       (30000, 128, 1e8), (3000, 100, 1e4), (800, 256, 1e5),
                                       (1000, 1, 1.0)])
def test_oblique_tridiagonal(scqr, m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(3, m + n))
    d, o = synth.tridiag_b(m, seed=synth.seed_for(3, 7 * n))
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), B=B, schedule="adaptive")
    assert info.status == scqr.OK, info
    Qh, Rh = host(Q), host(R)
    assert accuracy.orthogonality(Qh, (d, o))[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
    assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)
    # ||B||_2 bound and the first shift against the oracle's formula on the exact ||X||_2^2
    bn = oracle.gershgorin_tridiag(d, o)
    assert info.bnorm == pytest.approx(bn, rel=1e-15)
    lam = oracle.lambda_max(oracle.gram(X))
    s_exact = oracle.shift(m, n, lam, bnorm=bn, oblique=True)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-12)
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, tridiag=(d, o))
    assert ro.status == oracle.OK
    if kappa <= 1e10:
        assert ro.passes == info.passes
    if kappa <= 1e6:
        assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)
        assert np.max(np.abs(Qh - ro.Q)) <= 1e-10


def test_oblique_identity_b_matches_euclidean_with_same_shift(scqr):
    # B = I: every B-Gram is the Euclidean Gram; with the same (custom) shift formula the two
    # paths give the same factors up to rounding (their Grams are summed in different orders,
    # so the shifts and factors agree to about u and kappa u)
    m, n = 10000, 24
    X = synth.randsvd(m, n, 1e4, seed=93)
    Xd = torch.from_numpy(X).cuda()
    B = (torch.ones(m, dtype=torch.float64, device="cuda"), torch.zeros(m - 1, dtype=torch.float64, device="cuda"))
    Qb, Rb, ib = scqr.qr(Xd, B=B, shift="custom", custom_alpha=1e-10)
    Qe, Re, ie = scqr.qr(Xd, shift="custom", custom_alpha=1e-10)
    assert ib.status == ie.status == scqr.OK and ib.passes == ie.passes
    assert ib.shift[0] == pytest.approx(ie.shift[0], rel=1e-13)
    assert torch.linalg.norm(Rb - Re) <= 1e-11 * torch.linalg.norm(Re)
    assert torch.max(torch.abs(Qb - Qe)) <= 1e-11


def test_oblique_user_bnorm(scqr):
    m, n = 6000, 16
    X = synth.randsvd(m, n, 1e7, seed=94)
    d, o = synth.tridiag_b(m, seed=95)
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    _, _, info = scqr.qr(torch.from_numpy(X).cuda(), B=B, bnorm=2000.0)
    assert info.status == scqr.OK and info.bnorm == 2000.0
    lam = oracle.lambda_max(oracle.gram(X))
    s_exact = oracle.shift(m, n, lam, bnorm=2000.0, oblique=True)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-12)


@pytest.mark.parametrize("m,n,kappa", [(64, 64, 1e3), (65, 65, 1e3), (100, 100, 1e4), (4097, 128, 1e10),
                                       (20000, 96, 1e12), (130_000, 128, 1e13)])
def test_oblique_fused_pass_gram_replay(scqr, m, n, kappa):
    """Passes after the first form Q^T B Q of the Q they just wrote.  Replayed pass by pass: the
    traced B-Gram of pass p >= 2 agrees with the oracle's tridiagonal Gram of the replayed Q (the
    substitution entry point, bitwise the pass's Q) within 2 gamma_{m+3} |Q|^T |B| |Q|, with
    shapes of one, two and many 64-row panels, and the last replayed Q equals the factorization's
    Q bit for bit."""
    U = 2.0 ** -53
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(3, 5 * m + n))
    d, o = synth.tridiag_b(m, seed=synth.seed_for(3, 11 * n))
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), B=B, schedule="adaptive", trace=True)
    assert info.status == scqr.OK, info
    tr = info.trace.cpu().numpy()
    Qd = torch.from_numpy(X).cuda()
    g = (m + 3) * U / (1 - (m + 3) * U)
    for p in range(info.passes):
        if p >= 1:
            Qh = host(Qd)
            Go = oracle.gram_tridiag(Qh, d, o)
            absb = oracle.gram_tridiag(np.abs(Qh), np.abs(d), np.abs(o))
            assert np.all(np.abs(tr[p, 0] - Go) <= 2 * g * absb + 1e-300), f"B-Gram pass {p + 1}"
            np.testing.assert_array_equal(tr[p, 0], tr[p, 0].T)
        Qd = scqr.trsm(Qd, torch.from_numpy(np.ascontiguousarray(tr[p, 1])).cuda())
    np.testing.assert_array_equal(host(Qd), host(Q))
    Qh, Rh = host(Q), host(R)
    assert accuracy.orthogonality(Qh, (d, o))[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
