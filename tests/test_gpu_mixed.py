"""GPU parity of the FP32-first option: the Gram of pass 1 in binary32 MFMA (binary64 sums of
binary32 chains of k rows: k = 32 up to n = 64, 64 up to n = 128, 16 beyond), the binary32
shift s32 = 11((k + 2) n u32 + n(n+1) u) ||X||_2^2, every later step in binary64, and the
fall-back to an all-binary64 first pass when s32 > ||X||_2^2 / 100, the first Cholesky breaks
down, or the binary32 Gram is not finite (X finite in binary64 but beyond the binary32 range).

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
    k = oracle.f32_chain_rows(n)
    G32 = info.trace[0, 0].cpu().numpy()
    Ge = oracle.gram(X)
    absg = np.abs(X).T @ np.abs(X)
    assert np.all(np.abs(G32 - Ge) <= (k + 2) * U32 * absg + 1e-300)
    lam = np.linalg.eigvalsh(G32)[-1]
    s_exact = oracle.shift_f32(n, k, lam)
    assert s_exact * (1 - 1e-4) <= info.shift[0] <= s_exact * (1 + 1e-12)
    Qh, Rh = host(Q), host(R)
    assert accuracy.orthogonality(Qh)[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1)
    assert ro.fell_back == 0 and ro.passes == info.passes
    if kappa <= 1e6:
        assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)


@pytest.mark.parametrize("m,n,kappa", [(30000, 16, 1e7), (50000, 32, 1e8), (20000, 64, 1e6),
                                       (30000, 128, 1e7), (8000, 256, 1e6)])
def test_fp32_first_kappa_reduction_closed_form(scqr, m, n, kappa):
    # the GPU's binary32 first factor reduces kappa as the shift predicts (Section 4.1, with s32):
    # kappa(X R1^{-1}) = sqrt(sigma_n^2 + s32) / (sigma_n sqrt(1 + s32)) for ||X||_2 = 1, within
    # 10% (the binary32 Gram's error is at most s32 / 11)
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(6, 7 * m + n))
    Xd = torch.from_numpy(X).cuda()
    Q, R, info = scqr.qr(Xd, precision="fp32_first", trace=True)
    assert info.fell_back_fp64 == 0 and info.shifted_mask & 1
    s32 = info.shift[0]
    sv = np.linalg.svd(X, compute_uv=False)
    exact = (sv[0] / np.sqrt(sv[0] ** 2 + s32)) / (sv[-1] / np.sqrt(sv[-1] ** 2 + s32))
    Q1 = host(scqr.trsm(Xd, info.trace[0, 1].contiguous()))
    assert abs(accuracy.cond2(Q1) / exact - 1) < 0.10


def test_fp32_first_large_kappa_needs_continuation(scqr):
    # kappa(Q^(1)) ~ sqrt(alpha32) kappa exceeds u^{-1/2}: the binary64 passes that follow
    # continue with shifted passes (Algorithm 2) and still reach the invariants
    X = synth.randsvd(40000, 32, 1e13, seed=91)
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), precision="fp32_first")
    assert info.status == scqr.OK and info.fell_back_fp64 == 0
    assert info.passes >= 3
    assert accuracy.orthogonality(host(Q))[0] <= 1e-13
    assert accuracy.residual(X, host(Q), host(R)) <= 1e-13


@pytest.mark.parametrize("n,scale", [(16, 1e21), (64, 1e21), (128, 1e21), (256, 1e21), (64, 1.0)])
def test_fp32_first_falls_back_bitwise(scqr, n, scale):
    # X scaled by 1e21 is finite in binary64 but its binary32 Gram overflows: pass 1 is redone in
    # binary64 (the oracle's emulation decides the same), and the result is bitwise the all-binary64
    # one.  scale 1: the first Cholesky is forced to break down, the other fall-back route
    X = synth.randsvd(3000, n, 1e5, seed=92 + n) * scale
    Xd = torch.from_numpy(X).cuda()
    force = 1 if scale == 1.0 else 0
    Q32, R32, i32 = scqr.qr(Xd, precision="fp32_first", debug_force_breakdown_pass=force)
    Q64, R64, i64 = scqr.qr(Xd)
    assert i32.status == scqr.OK and i32.fell_back_fp64 == 1
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1, force_breakdown_pass=force)
    assert ro.fell_back == 1 and ro.status == oracle.OK
    assert torch.equal(Q32, Q64) and torch.equal(R32, R64)
    assert i32.passes == i64.passes
    assert accuracy.orthogonality(host(Q32))[0] <= 1e-13


def test_fp32_first_kept_at_the_widest_class(scqr):
    # with 16-row binary32 chains at n = 256 the binary32 shift stays below ||X||_2^2 / 100, so
    # the binary32 pass is kept there as at every other width
    assert oracle.shift_f32(256, oracle.f32_chain_rows(256), 1.0) < 0.01
    assert oracle.shift_f32(128, oracle.f32_chain_rows(128), 1.0) < 0.01
    X = synth.randsvd(3000, 256, 1e5, seed=93)
    Q, R, info = scqr.qr(torch.from_numpy(X).cuda(), precision="fp32_first")
    assert info.status == scqr.OK and info.fell_back_fp64 == 0
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1)
    assert ro.fell_back == 0 and ro.passes == info.passes
    assert accuracy.orthogonality(host(Q))[0] <= 1e-13
