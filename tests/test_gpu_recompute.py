"""GPU tests of the minimum-traffic passes (option ``recompute``, n <= 32, B = I).

Each pass before the last reads X, recomputes the previous iterate Q_{k-1} = X R~_1^{-1} ...
R~_{k-1}^{-1} through the same blocked row-wise substitution the stored passes apply one pass at
a time, and writes nothing but its Gram; only the last pass writes Q.  Since the recomputed
iterate is formed by the same operations in the same order, the factorization must equal the
default (stored) one bit for bit: Q, R, every per-pass Gram and factor of the trace, the
shifts, masks and pass count.  The oracle comparisons of the default path therefore carry over;
some are repeated here on the recomputed result (pass counts, factors at kappa <= 1e6, the
paper's invariants ||Q^T Q - I||_2 and ||X - QR||_F / ||X||_F <= 1e-13).
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def same_info(a, b):
    assert (a.status, a.passes, a.shifted_mask, a.breakdown_mask, a.fell_back_fp64) == \
        (b.status, b.passes, b.shifted_mask, b.breakdown_mask, b.fell_back_fp64)
    assert list(a.shift) == list(b.shift) and list(a.norm2sq) == list(b.norm2sq)
    assert list(a.gram_dev) == list(b.gram_dev) and a.omega_fro == b.omega_fro


CASES = [(4099, 1, 1.0, "adaptive"), (100003, 7, 1e8, "fixed3"), (20000, 16, 1e15, "adaptive"),
         (65537, 17, 1e12, "adaptive"), (30000, 31, 1e10, "iterated"), (50000, 32, 1e15, "adaptive"),
         (32, 32, 1e4, "fixed3"), (12345, 24, 1e5, "cholqr2"), (1000, 2, 1e15, "adaptive"),
         (777, 9, 1e13, "fixed3")]


@pytest.mark.parametrize("m,n,kappa,schedule", CASES)
def test_recompute_equals_stored(scqr, m, n, kappa, schedule):
    Xh = synth.randsvd(m, n, kappa, seed=synth.seed_for(9, m + n))
    X = dev(Xh)
    Qs, Rs, i_s = scqr.qr(X, schedule=schedule, trace=True)
    Qm, Rm, i_m = scqr.qr(X, schedule=schedule, trace=True, recompute=True)
    assert i_s.status == scqr.OK, i_s
    same_info(i_m, i_s)
    assert torch.equal(Qm, Qs) and torch.equal(Rm, Rs)
    assert torch.equal(i_m.trace, i_s.trace)
    np.testing.assert_array_equal(host(X), Xh)  # X is only read
    print(f"m={m} n={n} kappa={kappa:.0e} {schedule}: {i_m.passes} passes")


@pytest.mark.parametrize("m,n,kappa", [(20000, 16, 1e15), (5000, 17, 1e10), (40000, 32, 1e6),
                                       (3001, 5, 1e3)])
def test_recompute_against_oracle(scqr, m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(9, 3 * m + n))
    Q, R, info = scqr.qr(dev(X), schedule="adaptive", recompute=True)
    assert info.status == scqr.OK
    Qh, Rh = host(Q), host(R)
    ro = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    if kappa <= 1e12:  # below that the breakdown decisions are far from rounding
        assert ro.passes == info.passes and ro.shifted_mask == info.shifted_mask
    if kappa <= 1e6:
        assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R)
        assert np.max(np.abs(Qh - ro.Q)) <= 1e-10
    assert accuracy.orthogonality(Qh)[0] <= 1e-13
    assert accuracy.residual(X, Qh, Rh) <= 1e-13
    assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)


@pytest.mark.parametrize("n", [8, 30, 32])
def test_recompute_in_place_and_strided(scqr, n):
    m = 30011
    Xh = synth.randsvd(m, n, 1e12, seed=synth.seed_for(9, 7 * n))
    Qs, Rs, i_s = scqr.qr(dev(Xh))
    Xd = dev(Xh)
    Q, R, info = scqr.qr(Xd, inplace=True, recompute=True)
    assert info.status == scqr.OK and Q.data_ptr() == Xd.data_ptr()
    assert torch.equal(Q, Qs) and torch.equal(R, Rs)
    # X as a column block of a wider matrix (leading dimension n + 5, odd for odd n)
    W = torch.zeros((m, n + 5), dtype=torch.float64, device="cuda")
    W[:, 2:2 + n] = dev(Xh)
    Q2, R2, _ = scqr.qr(W[:, 2:2 + n], recompute=True)
    assert torch.equal(Q2, Qs) and torch.equal(R2, Rs)


def test_recompute_final_gram_and_fp32_first(scqr):
    X = dev(synth.randsvd(50000, 32, 1e11, seed=synth.seed_for(9, 1)))
    Qs, Rs, i_s = scqr.qr(X, final_gram=True)
    Qm, Rm, i_m = scqr.qr(X, final_gram=True, recompute=True)
    same_info(i_m, i_s)
    assert torch.equal(Qm, Qs) and torch.equal(Rm, Rs) and i_m.omega_fro <= 1e-13
    X = dev(synth.randsvd(60000, 20, 1e4, seed=synth.seed_for(9, 2)))
    Qs, Rs, i_s = scqr.qr(X, precision="fp32_first")
    Qm, Rm, i_m = scqr.qr(X, precision="fp32_first", recompute=True)
    same_info(i_m, i_s)
    assert torch.equal(Qm, Qs) and torch.equal(Rm, Rs)


def test_recompute_breakdown_leaves_x_unwritten(scqr):
    # a breakdown stops the schedule before the last pass, so an in-place call leaves X as it
    # was (the stored passes would have overwritten it with the first pass's Q)
    Xh = synth.randsvd(2000, 6, 1e3, seed=19)
    Xh[:, 5] = 0.0  # a zero pivot whatever the summation order
    Xd = dev(Xh)
    _, _, info = scqr.qr(Xd, inplace=True, schedule="fixed3", debug_zero_shift=True, recompute=True,
                         check="status")
    assert info.status == scqr.E_BREAKDOWN
    np.testing.assert_array_equal(host(Xd), Xh)
    Xh = synth.randsvd(3000, 16, 1e3, seed=16)
    _, _, info = scqr.qr(dev(Xh), schedule="fixed3", debug_force_breakdown_pass=3, recompute=True,
                         check="status")
    assert info.status == scqr.E_BREAKDOWN and info.passes == 2 and info.breakdown_mask == 4


@pytest.mark.slow
@pytest.mark.parametrize("n,kappa", [(32, 1e15), (16, 1e8)])
def test_recompute_full_size(scqr, n, kappa):
    # the minimum-traffic workload: 2^23 rows (2 GiB at n = 32), adaptive schedule
    m = 1 << 23
    X = dev(synth.randsvd(m, n, kappa, seed=synth.seed_for(9, n)))
    Qs, Rs, i_s = scqr.qr(X, final_gram=True)
    Qm, Rm, i_m = scqr.qr(X, final_gram=True, recompute=True)
    assert i_s.status == scqr.OK
    same_info(i_m, i_s)
    assert torch.equal(Qm, Qs) and torch.equal(Rm, Rs)
    assert i_m.omega_fro <= 1e-13
    print(f"m=2^23 n={n} kappa={kappa:.0e}: {i_m.passes} passes, omega_F {i_m.omega_fro:.2e}")
