"""End-to-end pins of the oracle's shifted Cholesky QR drivers (CPU only): a textbook
Householder QR on tiny inputs, closed forms, the values printed in Tables 1-3, the paper's
bounds (Lemma 1, Lemma 3, Theorem on shiftedCholeskyQR3) and invariant sweeps."""
import json
import os

import numpy as np
import pytest

import accuracy
import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
U = 2.0 ** -53


def householder_qr(X):
    """Textbook Householder QR (reflect column k onto -sign(x_kk)||x|| e_k), thin Q and R,
    then signs normalised so that diag(R) > 0.  Written independently of the oracle."""
    A = np.array(X, dtype=np.float64, copy=True)
    m, n = A.shape
    vs = []
    for k in range(n):
        x = A[k:, k].copy()
        nx = np.sqrt(np.sum(x * x))
        alpha = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] -= alpha
        nv = np.sqrt(np.sum(v * v))
        if nv > 0:
            v /= nv
            A[k:, k:] -= 2.0 * np.outer(v, v @ A[k:, k:])
        vs.append(v)
    R = np.triu(A[:n, :n])
    Q = np.zeros((m, n))
    Q[:n, :n] = np.eye(n)
    for k in reversed(range(n)):
        v = vs[k]
        Q[k:, :] -= 2.0 * np.outer(v, v @ Q[k:, :])
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, d[:, None] * R


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------- Householder cross-check
@pytest.mark.parametrize("m,n,kappa", [(8, 1, 1.0), (16, 4, 1e2), (40, 8, 1e4), (64, 8, 1e6),
                                       (9, 9, 1e3)])
@pytest.mark.parametrize("schedule", [oracle.FIXED3, oracle.ADAPTIVE, oracle.ITERATED])
def test_matches_householder_on_tiny_inputs(m, n, kappa, schedule):
    X = synth.randsvd(m, n, kappa, seed=1000 + m + n)
    r = oracle.scqr(X, schedule=schedule)
    assert r.status == oracle.OK
    Qh, Rh = householder_qr(X)
    tol = 50 * max(kappa, 1.0) * n * U
    assert relerr(r.R, Rh) <= tol
    assert np.max(np.abs(r.Q - Qh)) <= tol * 10
    assert np.all(np.diag(r.R) > 0)
    assert np.all(np.tril(r.R, -1) == 0)


# ---------------------------------------------------------------- closed forms
def test_single_column_closed_form():
    x = synth.gaussian((500, 1), 5)
    r = oracle.scqr(x)
    nrm = np.sqrt(np.sum(x * x))
    assert abs(r.R[0, 0] - nrm) <= 4 * U * nrm
    assert np.max(np.abs(r.Q - x / nrm)) <= 8 * U * np.max(np.abs(x / nrm))


def test_orthogonal_columns_give_diagonal_r():
    rng = np.random.default_rng(6)
    W, _ = np.linalg.qr(rng.standard_normal((300, 6)))
    norms = np.array([1.0, 3.0, 0.5, 10.0, 2.0, 7.0])
    r = oracle.scqr(W * norms)
    np.testing.assert_allclose(np.diag(r.R), norms, rtol=1e-13)
    assert np.max(np.abs(np.triu(r.R, 1))) <= 1e-13 * norms.max()


def test_stacked_triangular_input():
    rng = np.random.default_rng(7)
    n = 6
    R0 = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
    X = np.vstack([R0, np.zeros((30, n))])
    r = oracle.scqr(X)
    assert relerr(r.R, R0) <= 1e-14
    E = np.zeros((36, n))
    E[:n] = np.eye(n)
    assert np.max(np.abs(r.Q - E)) <= 1e-14


# ---------------------------------------------------------------- Tables 1 and 2
@pytest.mark.parametrize("tab", ["table1", "table2"])
def test_tables_1_2(tab):
    t = GOLD[tab]
    X = synth.randsvd(t["m"], t["n"], t["kappa"], seed=synth.seed_for(90, 1 if tab == "table1" else 2))
    r = oracle.scqr(X, schedule=oracle.FIXED3, history=True)
    assert r.status == oracle.OK and r.passes == 3 and r.shifted_mask == 1
    Q = X.copy()
    kap, om = [], []
    for Rt in r.rts:
        Q = oracle.trsm_rows(Q, Rt)
        kap.append(accuracy.cond2(Q))
        om.append(accuracy.orthogonality(Q)[0])
    assert abs(kap[0] / t["kappa_q"][0] - 1) < 0.10
    assert 1.0 <= kap[1] < 1.1 and kap[2] < 1.0 + 1e-12
    assert 0.5 < om[0] < 1.5
    assert t["omega2"][1] / 30 < om[1] < t["omega2"][1] * 30
    assert om[2] < 10 * t["omega2"][2]
    np.testing.assert_array_equal(Q, r.Q)
    # the adaptive reading stops after the same three passes (last input Gram near I)
    ra = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert ra.status == oracle.OK and ra.passes == 3
    np.testing.assert_array_equal(ra.Q, r.Q)


# ---------------------------------------------------------------- Table 3 (oblique, dense B)
def b_measure(Q, B):
    lam = np.linalg.eigvalsh(Q.T @ B @ Q)[0]
    return np.linalg.norm(Q, 2) * np.sqrt(np.linalg.norm(B, 2)) / np.sqrt(lam)


def test_table_3_dense_b():
    t = GOLD["table3"]
    m, n = t["m"], t["n"]
    X = synth.randsvd(m, n, t["kappa_x"], seed=synth.seed_for(90, 3))
    B = synth.dense_spd_b(m, t["kappa_b"], seed=synth.seed_for(90, 4))
    r = oracle.scqr(X, B=B, history=True)
    assert r.status == oracle.OK and r.passes == 3
    Q = X.copy()
    meas, om = [], []
    for Rt in r.rts:
        Q = oracle.trsm_rows(Q, Rt)
        meas.append(b_measure(Q, B))
        om.append(np.linalg.norm(Q.T @ B @ Q - np.eye(n), 2))
    assert t["measure_q"][0] / 3 < meas[0] < t["measure_q"][0] * 3
    assert t["measure_q"][1] / 3 < meas[1] < t["measure_q"][1] * 3
    assert abs(meas[2] / meas[1] - 1) < 0.2
    assert 0.5 < om[0] < 1.5 and om[1] < 0.5
    assert om[2] < 10 * t["omegaB2"][2]
    assert accuracy.residual(X, r.Q, r.R) < 1e-15


def test_oblique_identity_b_equals_euclidean_bitwise():
    X = synth.randsvd(500, 12, 1e9, seed=21)
    a = 1e-9
    r1 = oracle.scqr(X, shift_mode=oracle.SHIFT_CUSTOM, custom_alpha=a)
    r2 = oracle.scqr(X, tridiag=(np.ones(500), np.zeros(499)), shift_mode=oracle.SHIFT_CUSTOM,
                     custom_alpha=a)
    np.testing.assert_array_equal(r1.Q, r2.Q)
    np.testing.assert_array_equal(r1.R, r2.R)


def test_oblique_tridiag_b_orthogonality():
    m, n = 3000, 16
    X = synth.randsvd(m, n, 1e10, seed=22)
    d, o = synth.tridiag_b(m, seed=23)
    r = oracle.scqr(X, tridiag=(d, o), schedule=oracle.ADAPTIVE)
    assert r.status == oracle.OK
    om2, _ = accuracy.orthogonality(r.Q, tridiag=(d, o))
    assert om2 < 1e-13
    assert accuracy.residual(X, r.Q, r.R) < 1e-14


# ---------------------------------------------------------------- bounds of Section 3 and 4
@pytest.mark.parametrize("kappa", [1e8, 1e11, 1e14])
def test_lemma1_lemma3_after_shifted_pass(kappa):
    m, n = 800, 20
    X = synth.randsvd(m, n, kappa, seed=31)
    r = oracle.scqr(X, schedule=oracle.FIXED3, history=True)
    Q1 = oracle.trsm_rows(X, r.rts[0])
    G = accuracy.gram(Q1)
    assert np.max(np.abs(np.linalg.eigvalsh(G - np.eye(n)))) < 2.0          # Lemma 1
    assert np.linalg.norm(Q1, 2) < np.sqrt(3.0)
    res = np.linalg.norm(Q1 @ r.rts[0] - X) / np.linalg.norm(X, 2)           # Lemma 3
    assert res <= 2 * n * n * U
    # exact-arithmetic condition number of X R^{-1}: sqrt(sigma_n^2 + s) / (sigma_n sqrt(1 + s))
    s = r.shifts[0]
    sn = 1.0 / kappa
    predicted = np.sqrt(sn ** 2 + s) / (sn * np.sqrt(1 + s))
    assert abs(accuracy.cond2(Q1) / predicted - 1) < 0.25


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e9, 1.5e10])
def test_theorem_bounds_within_guarantee(kappa):
    m, n = 600, 10
    guarantee = 1.0 / (U * 96 * (m * n + n * (n + 1)))
    assert kappa <= guarantee
    X = synth.randsvd(m, n, kappa, seed=32)
    r = oracle.scqr(X, schedule=oracle.FIXED3)
    assert r.status == oracle.OK
    _, omf = accuracy.orthogonality(r.Q)
    assert omf <= 6 * (m * n + n * (n + 1)) * U
    res = np.linalg.norm(r.Q @ r.R - X) / np.linalg.norm(X, 2)
    assert res <= 15 * n * n * U


def test_cholqr2_when_kappa_small():
    X = synth.randsvd(2000, 20, 1e5, seed=33)
    r2 = oracle.scqr(X, schedule=oracle.CHOLQR2)
    ri = oracle.scqr(X, schedule=oracle.ITERATED)
    assert r2.status == ri.status == oracle.OK and r2.passes == ri.passes == 2
    np.testing.assert_array_equal(r2.Q, ri.Q)
    assert ri.shifted_mask == 0 and ri.breakdown_mask == 0
    assert accuracy.orthogonality(r2.Q)[0] < 1e-14


# ---------------------------------------------------------------- sweeps (Figures 4-6)
@pytest.mark.parametrize("kappa", [1e1, 1e4, 1e8, 1e10, 1e12, 1e13, 1e14, 1e15])
def test_sweep_kappa_orthogonality_and_residual_order_u(kappa):
    m, n = 300, 10
    X = synth.randsvd(m, n, kappa, seed=41)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert r.status == oracle.OK
    # the shifted Cholesky never breaks down up to kappa ~ 1/u (Section 4.1)
    assert r.breakdown_mask & 1 == 0
    om2, _ = accuracy.orthogonality(r.Q)
    assert om2 < 1e-14
    assert accuracy.residual(X, r.Q, r.R) < 1e-15


@pytest.mark.parametrize("m", [1000, 4000, 10000])
def test_sweep_m(m):
    X = synth.randsvd(m, 50, 1e12, seed=42)
    r = oracle.scqr(X)
    assert r.status == oracle.OK
    assert accuracy.orthogonality(r.Q)[0] < 1e-14
    assert accuracy.residual(X, r.Q, r.R) < 1e-15


@pytest.mark.parametrize("n", [10, 50, 150])
def test_sweep_n(n):
    X = synth.randsvd(1000, n, 1e12, seed=43)
    r = oracle.scqr(X)
    assert r.status == oracle.OK
    assert accuracy.orthogonality(r.Q)[0] < 1e-13
    assert accuracy.residual(X, r.Q, r.R) < 1e-15


@pytest.mark.parametrize("kx,kb", [(1e4, 1e10), (1e8, 1e10), (1e10, 1e8), (1e10, 1e12)])
def test_sweep_oblique_dense(kx, kb):
    m, n = 300, 20
    X = synth.randsvd(m, n, kx, seed=44)
    B = synth.dense_spd_b(m, kb, seed=45)
    r = oracle.scqr(X, B=B, schedule=oracle.ADAPTIVE)
    assert r.status == oracle.OK
    om = np.linalg.norm(r.Q.T @ B @ r.Q - np.eye(n), 2)
    # Theorem (oblique): ||Q^T B Q - I||_F <= 8 [m sqrt(mn) u + n(n+1) u] kappa(B); the paper
    # calls the kappa(B) dependence a large overestimate, which the test confirms.
    assert om <= 8 * (m * np.sqrt(m * n) + n * (n + 1)) * U * kb
    assert om < 1e-11
    assert accuracy.residual(X, r.Q, r.R) < 1e-14


# ---------------------------------------------------------------- adaptive continuation
def test_adaptive_reaches_kappa_one_over_u_with_extra_passes():
    m, n = 20000, 32
    X = synth.randsvd(m, n, 1e15, seed=51)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, max_passes=8)
    assert r.status == oracle.OK and r.passes >= 3
    assert accuracy.orthogonality(r.Q)[0] < 1e-13
    assert accuracy.residual(X, r.Q, r.R) < 1e-14


@pytest.mark.parametrize("kappa", [1e12, 1e15])
def test_small_shift_option(kappa):
    # s = u ||X||_2^2 (remark after Table 3): better reduction, no guarantee against breakdown
    X = synth.randsvd(1000, 50, kappa, seed=52)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, shift_mode=oracle.SHIFT_SMALL, history=True)
    assert r.shifts[0] == U * r.norm2sq[0]
    assert r.status in (oracle.OK, oracle.BREAKDOWN)
    if r.status == oracle.OK:
        assert accuracy.orthogonality(r.Q)[0] < 1e-13
        Q1 = oracle.trsm_rows(X, r.rts[0])
        assert accuracy.cond2(Q1) < 1e-6 * kappa
    else:
        assert r.breakdown_mask & 1 and r.passes == 0


def test_fro_shift_is_larger():
    X = synth.randsvd(1000, 20, 1e10, seed=53)
    rp = oracle.scqr(X, history=True)
    rf = oracle.scqr(X, shift_mode=oracle.SHIFT_FRO, history=True)
    assert rf.shifts[0] > rp.shifts[0]
    assert abs(rf.norm2sq[0] - np.sum(X * X)) <= 1e-12 * rf.norm2sq[0]


def test_fp32_first_emulation():
    X = synth.randsvd(20000, 16, 1e6, seed=54)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1, f32_chain=64, history=True)
    assert r.status == oracle.OK and r.fell_back == 0
    assert r.shifts[0] == oracle.shift_f32(16, 64, r.norm2sq[0])
    assert accuracy.orthogonality(r.Q)[0] < 1e-13
    assert accuracy.residual(X, r.Q, r.R) < 1e-14
    # a binary32 shift above ||X||^2 / 100 (here n = 128 with 128-row chains) falls back to
    # the binary64 pass
    assert oracle.shift_f32(128, 128, 1.0) > 0.01
    Xb = synth.randsvd(2000, 128, 1e6, seed=55)
    rb = oracle.scqr(Xb, schedule=oracle.ADAPTIVE, precision=1, f32_chain=128)
    assert rb.fell_back == 1 and rb.status == oracle.OK


@pytest.mark.parametrize("m,n,kappa", [(20000, 16, 1e7), (20000, 32, 1e8), (8000, 64, 1e6),
                                       (5000, 100, 1e7), (3000, 200, 1e6)])
def test_fp32_first_kappa_reduction_closed_form(m, n, kappa):
    # The binary32 first pass reduces the condition number as the shifted Cholesky of an exact
    # Gram would (Section 4.1: kappa(X R^{-1}) = sqrt(sigma_n^2 + s) / (sigma_n sqrt(1 + s)) for
    # ||X||_2 = 1), with s the binary32 shift s32: the binary32 Gram's error is below s32 / 11,
    # so the first factor's kappa must match the closed form within 10%.  A dropped term of
    # s32 (the chain length k, u32, the n(n+1) u part) or a binary32 Cholesky would miss it.
    X = synth.randsvd(m, n, kappa, seed=synth.seed_for(6, 11 * m + n))
    k = oracle.f32_chain_rows(n)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1, history=True)
    assert r.status == oracle.OK and r.fell_back == 0 and r.shifted_mask & 1
    sv = np.linalg.svd(X, compute_uv=False)
    s32 = 11.0 * ((k + 2) * n * oracle.U32 + n * (n + 1) * U) * sv[0] ** 2
    assert abs(r.shifts[0] / s32 - 1) < 1e-6   # the power iteration is exact enough here
    exact = (sv[0] / np.sqrt(sv[0] ** 2 + s32)) / (sv[-1] / np.sqrt(sv[-1] ** 2 + s32))
    k1 = accuracy.cond2(oracle.trsm_rows(X, r.rts[0]))
    assert abs(k1 / exact - 1) < 0.10
    # sqrt(alpha32) kappa is the leading term of the closed form
    assert abs(k1 / (np.sqrt(s32) * kappa) - 1) < 0.15


def test_fp32_first_overflow_falls_back():
    # entries near 1e19 square beyond the binary32 range: the binary32 Gram is not finite and
    # pass 1 is redone in binary64, giving bitwise the all-binary64 factorization
    X = synth.randsvd(3000, 24, 1e5, seed=56) * 1e21
    r32 = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1)
    r64 = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert r32.status == oracle.OK and r32.fell_back == 1
    assert np.array_equal(r32.Q, r64.Q) and np.array_equal(r32.R, r64.R)
    # a non-finite X stays non-finite after the fall-back
    X[5, 3] = np.inf
    rn = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1)
    assert rn.status == oracle.NONFINITE and rn.fell_back == 1


# ---------------------------------------------------------------- failure handling
def test_forced_breakdown():
    X = synth.randsvd(500, 8, 1e3, seed=61)
    r = oracle.scqr(X, schedule=oracle.FIXED3, force_breakdown_pass=2)
    assert r.status == oracle.BREAKDOWN and r.breakdown_mask == 2
    ra = oracle.scqr(X, schedule=oracle.ADAPTIVE, force_breakdown_pass=2)
    assert ra.status == oracle.OK and ra.shifted_mask & 2 and ra.breakdown_mask == 2
    assert accuracy.orthogonality(ra.Q)[0] < 1e-14


def test_zero_matrix_breaks_down():
    r = oracle.scqr(np.zeros((50, 4)))
    assert r.status == oracle.BREAKDOWN


def test_nonfinite_input():
    X = synth.randsvd(50, 4, 10.0, seed=62)
    X[7, 2] = np.nan
    r = oracle.scqr(X)
    assert r.status == oracle.NONFINITE


def test_rank_deficient_reports_status():
    X = synth.randsvd(200, 6, 1e3, seed=63)
    X[:, 5] = X[:, 2]
    r = oracle.scqr(X, schedule=oracle.FIXED3, zero_shift=True)
    assert r.status == oracle.BREAKDOWN


def test_not_converged_cap():
    X = synth.randsvd(3000, 20, 1e15, seed=64)
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE, max_passes=2)
    assert r.status == oracle.NOT_CONVERGED and r.passes == 2


def test_invalid_shapes():
    r = oracle.scqr(np.zeros((3, 5)))
    assert r.status == oracle.INVALID


# ------------------------------------------- shift study of the remark after Table 3 (Figure shift_test)
SHIFT_STUDY = (1000, 50, 1e15)
SHIFT_STUDY_ALPHAS = [11 * (1000 * 50 + 50 * 51) * U, 1e-11, 1e-12, 1e-13, 1e-14, 1e-15]


def kappa_after_shifted_pass(sv, s):
    """Exact-arithmetic condition number of X R^{-1} with R^T R = X^T X + s I: the singular
    values of that factor are sigma_i / sqrt(sigma_i^2 + s), increasing in sigma_i."""
    return (sv[0] / np.sqrt(sv[0] ** 2 + s)) / (sv[-1] / np.sqrt(sv[-1] ** 2 + s))


def test_shift_study_kappa_of_first_factor():
    # m = 1000, n = 50, kappa = 1e15, the shift varied: kappa(Q^(1)) follows the closed form
    # above down to s = 1e-15 ||X||^2, stays within (eq:CNreduction), and the paper's shift
    # (about 6.4e-11 here) leaves it above what (eq:cholqr2gurantee) asks of CholeskyQR2.
    m, n, kappa = SHIFT_STUDY
    X = synth.randsvd(m, n, kappa, seed=61)
    sv = np.linalg.svd(X, compute_uv=False)
    need = 1.0 / (8 * np.sqrt((m * n + n * (n + 1)) * U))
    ks = []
    for a in SHIFT_STUDY_ALPHAS:
        r = oracle.scqr(X, schedule=oracle.FIXED3, shift_mode=oracle.SHIFT_CUSTOM, custom_alpha=a,
                        history=True)
        assert not r.breakdown_mask & 1
        s = r.shifts[0]
        assert s == a * r.norm2sq[0] and abs(r.norm2sq[0] / sv[0] ** 2 - 1) < 1e-10
        k = accuracy.cond2(oracle.trsm_rows(X, r.rts[0]))
        assert abs(k / kappa_after_shifted_pass(sv, s) - 1) < 0.05
        assert k <= 2 * np.sqrt(3) * np.sqrt(1 + a * (sv[0] / sv[-1]) ** 2)
        ks.append(k)
        # the two unshifted passes of Algorithm 3 go through when kappa(Q^(1)) is below u^{-1/2};
        # above it nothing is guaranteed (whether the second Cholesky breaks down is rounding)
        if k < 0.5 / np.sqrt(U):
            assert r.status == oracle.OK and r.passes == 3
            assert accuracy.orthogonality(r.Q)[0] < 1e-13
    assert ks[0] > need
    assert all(k1 > 2.5 * k2 for k1, k2 in zip(ks, ks[1:]))
    # the continuation (Algorithm 2) finishes from the paper's shift with extra passes
    r = oracle.scqr(X, schedule=oracle.ADAPTIVE)
    assert r.status == oracle.OK and r.passes > 3
    assert accuracy.orthogonality(r.Q)[0] < 1e-13


def test_shift_study_small_shift():
    # s = u ||X||_2^2: no guarantee against breakdown; without one, kappa(Q^(1)) <= u^{-1/2}
    m, n, kappa = SHIFT_STUDY
    X = synth.randsvd(m, n, kappa, seed=61)
    r = oracle.scqr(X, schedule=oracle.FIXED3, shift_mode=oracle.SHIFT_SMALL, history=True)
    assert r.shifts[0] == U * r.norm2sq[0]
    if r.breakdown_mask & 1:
        assert r.status == oracle.BREAKDOWN and r.passes == 0
    else:
        assert accuracy.cond2(oracle.trsm_rows(X, r.rts[0])) <= 1 / np.sqrt(U)
