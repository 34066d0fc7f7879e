"""Parity at the benchmark's full sizes, in the launch configuration bench.py times (a Plan per
shape, adaptive schedule, the paper's shift):

* m = 2^22, n = 64, kappa = 1e6: the factors match the oracle's full factorization
  (||R - R_orc||_F / ||R_orc||_F <= 1e-10, Q on sampled rows), invariants <= 1e-13;
* m = 2^22, n = 64, kappa = 1e15: the Gram of pass 1 is within the binary64 summation bound
  of the oracle's Gram of X, the first shift is equation (eq:finds2) on it, the invariants hold
  (the pass count at kappa ~ 1/u is reported: parity unpinned there);
* m = 10^6, n = 128, kappa = 1e13 with the tridiagonal B: ||Q^T B Q - I||_2 and the residual
  <= 1e-13, and the first shift is equation (eq:finds2B) with the Gershgorin bound of ||B||_2.
* beyond 2^32 elements (n = 64, 128, 256; 17 stacked copies of one (2^(28 - log2 n) + 37) x n matrix
  Y, kappa = 1e6; Euclidean and with a block-diagonal tridiagonal B): R = sqrt(17) R_Y of the
  oracle within 1e-10, sampled rows of Q in every copy
  (the last ones included) equal Q_Y / sqrt(17) of the oracle within 1e-10 and each other to rounding.
"""
import numpy as np
import pytest
import torch

import accuracy
import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
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


def test_full_size_kappa_1e6_matches_oracle(scqr):
    m, n = 1 << 22, 64
    X = synth.randsvd(m, n, 1e6, seed=synth.seed_for(1, 2))
    plan = scqr.Plan(m, n, "cuda", schedule="adaptive", shift="paper")
    Q, R = plan.run(torch.from_numpy(X).cuda())
    info = plan.read_info()
    assert info.status == scqr.OK
    Qh, Rh = host(Q), host(R)
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert ro.status == oracle.OK and ro.passes == info.passes
    assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)
    rows = np.random.default_rng(1).choice(m, 4096, replace=False)
    assert np.max(np.abs(Qh[rows] - ro.Q[rows])) <= 1e-10
    assert accuracy.orthogonality(Qh)[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13


def test_full_size_kappa_1e15_gram_shift_invariants(scqr):
    m, n = 1 << 22, 64
    X = synth.randsvd(m, n, 1e15, seed=synth.seed_for(1))
    Xd = torch.from_numpy(X).cuda()
    plan = scqr.Plan(m, n, "cuda", schedule="adaptive", shift="paper")
    Q, R = plan.run(Xd)
    info = plan.read_info()
    assert info.status == scqr.OK
    Qh, Rh = host(Q), host(R)
    om2, _ = accuracy.orthogonality(Qh)
    res = accuracy.residual(X, Qh, Rh)
    print(f"2^22 x 64, kappa 1e15: passes {info.passes}, shifted mask {info.shifted_mask}, "
          f"||Q^TQ-I||_2 = {om2:.2e}, residual = {res:.2e}")
    assert om2 <= 1e-13 and res <= 1e-13
    G = host(scqr.gram(Xd))
    Go = oracle.gram(X)
    gm = m * U / (1 - m * U)
    absg = np.abs(X).T @ np.abs(X)
    assert np.all(np.abs(G - Go) <= 2 * gm * absg)
    lam = np.linalg.eigvalsh(Go)[-1]
    s_exact = oracle.shift(m, n, lam)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-6)


def test_full_size_oblique(scqr):
    m, n = 1000000, 128
    X = synth.randsvd(m, n, 1e13, seed=synth.seed_for(2))
    d, o = synth.tridiag_b(m, seed=synth.seed_for(2, 1))
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    plan = scqr.Plan(m, n, "cuda", B=B, schedule="adaptive", shift="paper")
    Q, R = plan.run(torch.from_numpy(X).cuda())
    info = plan.read_info()
    assert info.status == scqr.OK
    Qh, Rh = host(Q), host(R)
    om2, _ = accuracy.orthogonality(Qh, (d, o))
    res = accuracy.residual(X, Qh, Rh)
    print(f"1e6 x 128 oblique, kappa 1e13: passes {info.passes}, ||Q^TBQ-I||_2 = {om2:.2e}, residual = {res:.2e}")
    assert om2 <= 1e-13 and res <= 1e-13
    bn = oracle.gershgorin_tridiag(d, o)
    assert info.bnorm == pytest.approx(bn, rel=1e-15)
    lam = oracle.lambda_max(oracle.gram(X))
    s_exact = oracle.shift(m, n, lam, bnorm=bn, oblique=True)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-6)


BIG = [((1 << 22) + 37, 64, 3), ((1 << 21) + 37, 128, 4), ((1 << 20) + 37, 256, 5)]


def _stacked_case(scqr, my, n, inst, oblique):
    # X = 17 stacked copies of Y (my x n, kappa = 1e6): about 4.56e9 elements, so the copies past
    # the 8th sit beyond 2^31 and the last one beyond 2^32 elements.  With B = diag(B_Y, ..., B_Y)
    # (tridiagonal, a zero off-diagonal entry between copies) X^T B X = 17 Y^T B_Y Y, so in exact
    # arithmetic R_X = sqrt(17) R_Y and every block of Q_X is Q_Y / sqrt(17); the row-wise
    # substitution treats equal rows alike, so the blocks of Q_X agree to rounding.
    c = 17
    m = c * my
    assert m * n > 1 << 32 and m < 1 << 31
    Y = synth.randsvd(my, n, 1e6, seed=synth.seed_for(1, inst))
    X = torch.from_numpy(Y).cuda().repeat(c, 1)
    assert X.shape == (m, n)
    Bd = By = None
    if oblique:
        d, o = synth.tridiag_b(my, seed=synth.seed_for(2, inst))
        By = (d, o)
        oX = np.concatenate([np.concatenate([o, [0.0]]) for _ in range(c - 1)] + [o])
        Bd = (torch.from_numpy(d).cuda().repeat(c), torch.from_numpy(oX).cuda())
        assert Bd[0].numel() == m and Bd[1].numel() == m - 1
    print(f"factorizing {m} x {n} ({m * n} elements), oblique {oblique}", flush=True)
    Q, R, info = scqr.qr(X, B=Bd)
    assert info.status == scqr.OK
    del X
    ro = oracle.scqr(Y, tridiag=By, schedule=oracle.ADAPTIVE)
    assert ro.status == oracle.OK
    sc = np.sqrt(float(c))
    Rh = host(R)
    rerr = np.linalg.norm(Rh - sc * ro.R) / np.linalg.norm(sc * ro.R)
    base = np.concatenate([[0, 1, my - 1], np.random.default_rng(3).choice(my, 61, replace=False)])
    rows = np.concatenate([k * my + base for k in range(c)])
    Qs = host(Q[torch.from_numpy(rows).cuda()]).reshape(c, base.size, n)
    qerr = np.max(np.abs(Qs[0] - ro.Q[base] / sc))
    spread = np.max(np.abs(Qs - Qs[0]))
    print(f"passes {info.passes} (oracle on Y {ro.passes}); ||R - sqrt(17) R_Y|| / ||.|| = {rerr:.2e}; "
          f"max |Q - Q_Y / sqrt(17)| = {qerr:.2e}; max spread over copies = {spread:.2e}", flush=True)
    assert rerr <= 1e-10
    assert qerr <= 1e-10
    assert spread <= 64 * U * np.max(np.abs(Qs[0]))
    assert np.abs(Qs[-1, 2]).max() > 0  # the last row of X was written


@pytest.mark.parametrize("my,n,inst", BIG)
def test_beyond_2_32_elements(scqr, my, n, inst):
    _stacked_case(scqr, my, n, inst, oblique=False)


@pytest.mark.parametrize("my,n,inst", BIG)
def test_beyond_2_32_elements_oblique(scqr, my, n, inst):
    _stacked_case(scqr, my, n, inst, oblique=True)
