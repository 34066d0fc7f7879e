"""Pins of the oracle's QR adjoint (CPU only): the n = 1 closed form, central finite
differences through the oracle's own forward pass, and torch's CPU autograd through a
sign-normalised Householder QR."""
import numpy as np
import pytest
import torch

import oracle
import synth


def loss_and_grad(X, dQ, dR):
    r = oracle.scqr(X)
    assert r.status == oracle.OK
    L = np.sum(dQ * r.Q) + np.sum(np.triu(dR) * r.R)
    return L, oracle.qr_backward(r.Q, r.R, dQ, dR), r


def test_n1_closed_form():
    x = synth.gaussian((300, 1), 1)
    dq = synth.gaussian((300, 1), 2)
    dr = np.array([[0.7]])
    r = oracle.scqr(x)
    q, rr = r.Q, r.R[0, 0]
    expect = dq / rr - q * (q[:, 0] @ dq[:, 0]) / rr + q * dr[0, 0]
    np.testing.assert_allclose(oracle.qr_backward(q, r.R, dq, dr), expect, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("m,n,kappa", [(64, 6, 10.0), (2048, 16, 1e2)])
def test_central_finite_differences(m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=100 + n)
    dQ, dR = synth.upstream_grads(m, n, seed=200 + n)
    _, G, _ = loss_and_grad(X, dQ, dR)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(8):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        Lp, _, _ = loss_and_grad(X + h * E, dQ, dR)
        Lm, _, _ = loss_and_grad(X - h * E, dQ, dR)
        fd = (Lp - Lm) / (2 * h)
        an = np.sum(G * E)
        assert abs(fd - an) <= 1e-5 * max(abs(an), np.linalg.norm(G) * 1e-3)


def test_against_torch_autograd_of_householder_qr():
    m, n = 500, 12
    X = synth.randsvd(m, n, 1e3, seed=300)
    dQ, dR = synth.upstream_grads(m, n, seed=301)
    Xt = torch.tensor(X, requires_grad=True)
    Qt, Rt = torch.linalg.qr(Xt)
    d = torch.sign(torch.diagonal(Rt)).detach()
    Qn, Rn = Qt * d, d[:, None] * Rt
    L = (Qn * torch.tensor(dQ)).sum() + (Rn * torch.tensor(dR)).sum()
    L.backward()
    _, G, _ = loss_and_grad(X, dQ, dR)
    np.testing.assert_allclose(G, Xt.grad.numpy(), rtol=1e-8, atol=1e-10)


def test_none_upstream_is_zero():
    X = synth.randsvd(200, 5, 10.0, seed=302)
    r = oracle.scqr(X)
    dQ, dR = synth.upstream_grads(200, 5, seed=303)
    z = np.zeros_like(dQ)
    np.testing.assert_array_equal(oracle.qr_backward(r.Q, r.R, None, dR),
                                  oracle.qr_backward(r.Q, r.R, z, dR))
    np.testing.assert_array_equal(oracle.qr_backward(r.Q, r.R, dQ, None),
                                  oracle.qr_backward(r.Q, r.R, dQ, np.zeros((5, 5))))
    # only the upper triangle of dR is read
    np.testing.assert_array_equal(oracle.qr_backward(r.Q, r.R, dQ, dR + np.tril(np.ones((5, 5)), -1)),
                                  oracle.qr_backward(r.Q, r.R, dQ, dR))
