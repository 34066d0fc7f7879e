"""GPU parity of the QR adjoint
    M = R dR^T - dQ^T Q,   dX = (dQ + Q copyltu(M)) R^{-T}
against the oracle's adjoint on the same (Q, R, dQ, dR), through the C ABI, plus the n = 1
closed form, zero (None) upstream gradients and central finite differences of
L = <dQ, Q> + <dR, R> through QRFunction (forward and backward on the GPU), and operands of
about 4.56e9 elements (beyond 2^32) built from 17 copies of one problem.

The two implementations compute the same formula in binary64 with different summation orders;
their difference is bounded by a small multiple of u kappa(R) ||dX||.
"""
import numpy as np
import pytest
import torch

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,n,kappa", [(5000, 16, 1e4), (3001, 64, 1e6), (4000, 100, 1e3),
                                       (2500, 128, 1e5), (1500, 256, 1e4), (777, 33, 10.0),
                                       (300, 1, 1.0)])
def test_backward_matches_oracle(scqr, m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(5, m + n))
    Q, R, info = scqr.qr(dev(X))
    assert info.status == scqr.OK
    dQ, dR = synth.upstream_grads(m, n, seed=synth.seed_for(5, 3 * n))
    dX = host(scqr.qr_backward(Q, R, dev(dQ), dev(dR)))
    ref = oracle.qr_backward(host(Q), host(R), dQ, dR)
    assert np.linalg.norm(dX - ref) <= 64 * n * U * kappa * np.linalg.norm(ref)


def test_backward_none_and_lower_triangle_ignored(scqr):
    m, n = 2000, 20
    X = synth.randsvd(m, n, 1e3, seed=401)
    Q, R, _ = scqr.qr(dev(X))
    dQ, dR = synth.upstream_grads(m, n, seed=402)
    Qh, Rh = host(Q), host(R)
    a = host(scqr.qr_backward(Q, R, None, dev(dR)))
    np.testing.assert_allclose(a, oracle.qr_backward(Qh, Rh, None, dR), rtol=0, atol=1e-11 * np.abs(a).max())
    b = host(scqr.qr_backward(Q, R, dev(dQ), None))
    np.testing.assert_allclose(b, oracle.qr_backward(Qh, Rh, dQ, None), rtol=0, atol=1e-11 * np.abs(b).max())
    # only the upper triangle of dR is read
    junk = dR + np.tril(np.full((n, n), 7.0), -1)
    c = host(scqr.qr_backward(Q, R, dev(dQ), dev(junk)))
    d = host(scqr.qr_backward(Q, R, dev(dQ), dev(dR)))
    np.testing.assert_array_equal(c, d)
    z = host(scqr.qr_backward(Q, R, None, None))
    assert np.all(z == 0.0)


def test_backward_n1_closed_form(scqr):
    x = synth.gaussian((4096, 1), 403)
    dq = synth.gaussian((4096, 1), 404)
    Q, R, _ = scqr.qr(dev(x))
    q, r = host(Q), host(R)[0, 0]
    expect = dq / r - q * (q[:, 0] @ dq[:, 0]) / r + q * 0.7
    got = host(scqr.qr_backward(Q, R, dev(dq), dev(np.array([[0.7]]))))
    np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-14)


def test_finite_differences_through_qrfunction(scqr):
    m, n = 2048, 16
    X = synth.randsvd(m, n, 1e2, seed=405)
    dQ, dR = synth.upstream_grads(m, n, seed=406)
    dQd, dRd = dev(dQ), dev(dR)
    Xd = dev(X).requires_grad_(True)
    Q, R = scqr.QRFunction.apply(Xd)
    L = (Q * dQd).sum() + (R * dRd).sum()
    L.backward()
    G = host(Xd.grad)

    def loss(Y):
        Qy, Ry, info = scqr.qr(dev(Y))
        assert info.status == scqr.OK
        return float((Qy * dQd).sum() + (Ry * dRd).sum())

    rng = np.random.default_rng(407)
    h = 1e-6
    for _ in range(8):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (loss(X + h * E) - loss(X - h * E)) / (2 * h)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-5 * max(abs(an), np.linalg.norm(G) * 1e-3)


@pytest.mark.slow
def test_backward_full_size(scqr):
    # 2^20 x 256, kappa = 1e8: forward (Algorithm 3) then the adjoint, against the oracle's
    # adjoint on the same Q and R
    m, n = 1 << 20, 256
    X = synth.randsvd(m, n, 1e8, seed=synth.seed_for(5))
    Q, R, info = scqr.qr(dev(X))
    assert info.status == scqr.OK
    dQ, dR = synth.upstream_grads(m, n, seed=synth.seed_for(5, 1))
    dX = host(scqr.qr_backward(Q, R, dev(dQ), dev(dR)))
    ref = oracle.qr_backward(host(Q), host(R), dQ, dR)
    err = np.linalg.norm(dX - ref) / np.linalg.norm(ref)
    print(f"full-size adjoint: ||dX - dX_orc||_F / ||dX_orc||_F = {err:.2e}")
    assert err <= 1e-6


@pytest.mark.slow
@pytest.mark.parametrize("my,n,inst", [((1 << 22) + 37, 64, 6), ((1 << 21) + 37, 128, 7),
                                       ((1 << 20) + 37, 256, 8)])
def test_backward_beyond_2_32_elements(scqr, my, n, inst):
    # 17 stacked copies, about 4.56e9 elements per m x n operand: Q = [Q_Y; ...] / sqrt(17),
    # R = sqrt(17) R_Y, dQ = [dQ_Y; ...], dR = dR_Y give M = sqrt(17) M_Y and every block of dX
    # equal to dX_Y / sqrt(17); the product with Q and the transposed solve are row-wise, so the
    # blocks agree to rounding.
    c = 17
    m = c * my
    assert m * n > 1 << 32 and m < 1 << 31
    sc = np.sqrt(float(c))
    Y = synth.randsvd(my, n, 1e6, seed=synth.seed_for(5, inst))
    ry = oracle.scqr(Y, schedule=oracle.ADAPTIVE)
    assert ry.status == oracle.OK
    dQy, dRy = synth.upstream_grads(my, n, seed=synth.seed_for(5, 10 + inst))
    ref = oracle.qr_backward(ry.Q, ry.R, dQy, dRy) / sc
    del Y
    Q = dev(ry.Q / sc).repeat(c, 1)
    dQ = dev(dQy).repeat(c, 1)
    print(f"adjoint at {m} x {n} ({m * n} elements)", flush=True)
    dX = scqr.qr_backward(Q, dev(sc * ry.R), dQ, dev(dRy))
    del Q, dQ
    base = np.concatenate([[0, 1, my - 1], np.random.default_rng(4).choice(my, 61, replace=False)])
    rows = np.concatenate([k * my + base for k in range(c)])
    dXs = host(dX[torch.from_numpy(rows).cuda()]).reshape(c, base.size, n)
    rel = np.linalg.norm(dXs[0] - ref[base]) / np.linalg.norm(ref[base])
    spread = np.max(np.abs(dXs - dXs[0]))
    print(f"||dX - dX_Y / sqrt(17)|| / ||.|| on sampled rows = {rel:.2e}; max spread over copies = "
          f"{spread:.2e}", flush=True)
    assert rel <= 64 * n * U * 1e6
    assert spread <= 64 * U * np.max(np.abs(dXs[0]))
    assert np.abs(dXs[-1, 2]).max() > 0  # the last row was written
