"""GPU parity of the FP32-first option: the Gram of pass 1 in binary32 MFMA (binary64 sums of
32-row binary32 chains), the binary32 shift s32 = 11((k + 2) n u32 + n(n+1) u) ||X||_2^2 with
k = 64, every later step in binary64, and the fall-back to an all-binary64 first pass when
s32 > ||X||_2^2 / 100 or the first Cholesky breaks down.

* The binary32 Gram is within the binary32 summation bound of the exact Gram of X (the oracle's
  binary64 Gram, itself within the binary64 bound).
* Its shift is equation (eq:finds2)'s form with the binary32 constants on that Gram, and the
  factorization meets the same final invariants as the binary64 path.
* The fall-back decision equals the oracle's emulation of the option, and after a fall-back
  the result is bitwise the all-binary64 result (the redo uses the binary64 kernels).
"""
import numpy as np
import pytest
import torch

import accuracy
import oracle
import synth

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def scqr():
    import paper_1809_11085_amd as s
    assert torch.cuda.is_available()
    s.lib()
    return s


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,n,kappa", [(20000, 16, 1e6), (50000, 32, 1e8), (4097, 64, 1e4),
                                       (30000, 128, 1e6), (1000, 17, 1e3)])
def test_fp32_first_gram_shift_and_invariants(scqr, m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(6, m + n))
    Xd = torch.from_numpy(X).cuda()
    Q, R, info = scqr.qr(Xd, precision="fp32_first", trace=True)
    assert info.status == scqr.OK, info
    assert info.fell_back_fp64 == 0
    G32 = info.trace[0, 0].cpu().numpy()
    Ge = oracle.gram(X)
    absg = np.abs(X).T @ np.abs(X)
    assert np.all(np.abs(G32 - Ge) <= (64 + 2) * U32 * absg + 1e-300)
    lam = np.linalg.eigvalsh(G32)[-1]
    s_exact = oracle.shift_f32(n, 64, lam)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-12)
    Qh, Rh = host(Q), host(R)
    assert accuracy.orthogonality(Qh)[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1, f32_chain=64)
    assert ro.fell_back == 0 and ro.passes == info.passes
    if kappa <= 1e6:
        assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)


def test_fp32_first_large_kappa_needs_continuation(scqr):
    # kappa(Q^(1)) ~ sqrt(alpha32) kappa exceeds u^{-1/2}: the binary64 passes that follow
    # continue with shifted passes (Algorithm 2) and still reach the invariants
    X = synth.randsvd(40000, 32, 1e13, seed=91)
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), precision="fp32_first")
    assert info.status == scqr.OK and info.fell_back_fp64 == 0
    assert info.passes >= 3
    assert accuracy.orthogonality(host(Q))[0] <= 1e-13
    assert accuracy.residual(X, host(Q), host(R)) <= 1e-13


def test_fp32_first_falls_back_bitwise(scqr):
    # n = 256: s32 = 11 * 66 * 256 * u32 ||X||^2 > ||X||^2 / 100, so pass 1 is redone in binary64
    X = synth.randsvd(3000, 256, 1e5, seed=92)
    Xd = torch.from_numpy(X).cuda()
    assert oracle.shift_f32(256, 64, 1.0) > 0.01
    Q32, R32, i32 = scqr.qr(Xd, precision="fp32_first")
    Q64, R64, i64 = scqr.qr(Xd)
    assert i32.status == scqr.OK and i32.fell_back_fp64 == 1
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1, f32_chain=64)
    assert ro.fell_back == 1
    assert torch.equal(Q32, Q64) and torch.equal(R32, R64)
    assert i32.passes == i64.passes
