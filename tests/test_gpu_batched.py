"""GPU parity of the batched factorization (one launch per width class and step) against the
oracle and against the single-instance path, through the C ABI.

* Every instance of an uneven batch meets the invariants of the paper (||Q^T Q - I||_2 and
  ||X - QR||_F / ||X||_F <= 1e-13, R upper triangular with positive diagonal), takes the same
  number of passes as the oracle for kappa <= 1e12 (nearer 1/u a borderline breakdown may go
  either way), and for kappa <= 1e6 its factors match the oracle's.
* Batched and single-instance calls run the same kernels on different row partitions, so they
  agree to rounding (not bitwise); two batched calls agree bitwise.
* The schedule is predicated per instance: a non-finite or rank-deficient instance reports its
  own status while the others complete.
"""
import numpy as np
import pytest
import torch

import accuracy
import oracle
import synth

pytestmark = pytest.mark.gpu

# (m, n, kappa): every width class, ragged m, n = 1, tall-thin and nearly square instances
BATCH = [(20000, 16, 1e12), (3000, 1, 1.0), (4097, 17, 1e5), (12345, 32, 1e14), (700, 40, 1e3),
         (33000, 64, 1e15), (65, 64, 1e6), (5000, 100, 1e9), (9000, 128, 1e13), (1500, 200, 1e4),
         (2049, 256, 1e6), (40000, 8, 1e8), (257, 255, 1e2), (18000, 48, 1e11), (1024, 128, 1e6),
         (100000, 16, 1e6)]


@pytest.fixture(scope="module")
def scqr():
    import paper_1809_11085_amd as s
    assert torch.cuda.is_available()
    s.lib()
    return s


@pytest.fixture(scope="module")
def batch_inputs():
    return [synth.randsvd(m, n, k, seed=synth.seed_for(4, i)) for i, (m, n, k) in enumerate(BATCH)]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_batched_matches_oracle(scqr, batch_inputs):
    Xs = [torch.from_numpy(X).cuda() for X in batch_inputs]
    Qs, Rs, infos = scqr.qr_batched(Xs, schedule="adaptive")
    for i, ((m, n, kappa), X) in enumerate(zip(BATCH, batch_inputs)):
        info = infos[i]
        assert info.status == scqr.OK, (i, info)
        Qh, Rh = host(Qs[i]), host(Rs[i])
        assert accuracy.orthogonality(Qh)[0] <= 1e-13, i
        assert accuracy.residual(X, Qh, Rh) <= 1e-13, i
        assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0), i
        ro = oracle.scqr(X, schedule=oracle.ADAPTIVE)
        if kappa <= 1e12:  # near 1/u a borderline breakdown may go either way (pass count unpinned)
            assert ro.passes == info.passes and ro.shifted_mask == info.shifted_mask, (i, ro.passes, info.passes)
        if kappa <= 1e6:
            assert np.linalg.norm(Rh - ro.R) <= 1e-10 * np.linalg.norm(ro.R), i
            assert np.max(np.abs(Qh - ro.Q)) <= 1e-10, i


def test_batched_vs_single_and_deterministic(scqr, batch_inputs):
    Xs = [torch.from_numpy(X).cuda() for X in batch_inputs]
    Q1, R1, i1 = scqr.qr_batched(Xs)
    Q2, R2, i2 = scqr.qr_batched(Xs)
    for i in range(len(Xs)):
        assert torch.equal(Q1[i], Q2[i]) and torch.equal(R1[i], R2[i])
        Qs, Rs, info = scqr.qr(Xs[i])
        kappa = BATCH[i][2]
        if kappa <= 1e12:
            assert info.passes == i1[i].passes and info.shifted_mask == i1[i].shifted_mask
        assert abs(info.shift[0] - i1[i].shift[0]) <= 1e-12 * max(info.shift[0], 1e-300)
        tol = max(1e-13, 64 * 2.0 ** -53 * kappa)
        assert torch.linalg.norm(R1[i] - Rs) <= tol * torch.linalg.norm(Rs), i


def test_batched_in_place_and_fixed3(scqr, batch_inputs):
    # instances with sqrt(alpha) kappa < u^{-1/2}, where Algorithm 3 alone completes
    Xs = [torch.from_numpy(batch_inputs[i]).cuda() for i in (0, 1, 2, 4, 6, 7)]
    ref_Q, ref_R, _ = scqr.qr_batched(Xs, schedule="fixed3")
    Xc = [X.clone() for X in Xs]
    Q, R, infos = scqr.qr_batched(Xc, inplace=True, schedule="fixed3")
    for i in range(len(Xs)):
        assert Q[i].data_ptr() == Xc[i].data_ptr()
        assert torch.equal(Q[i], ref_Q[i]) and torch.equal(R[i], ref_R[i])
        assert infos[i].status == scqr.OK and infos[i].passes == 3


def test_batched_per_instance_status(scqr):
    good = synth.randsvd(5000, 24, 1e8, seed=71)
    nan = synth.randsvd(3000, 24, 1e3, seed=72)
    nan[17, 5] = np.nan
    zero = np.zeros((2000, 33))
    big = synth.randsvd(8000, 70, 1e10, seed=73)
    Xs = [torch.from_numpy(a).cuda() for a in (good, nan, zero, big)]
    Qs, Rs, infos = scqr.qr_batched(Xs, check="status")
    assert infos[0].status == scqr.OK and infos[3].status == scqr.OK
    assert infos[1].status == scqr.E_NONFINITE
    assert infos[2].status == scqr.E_BREAKDOWN
    for i, X in ((0, good), (3, big)):
        assert accuracy.orthogonality(host(Qs[i]))[0] <= 1e-13
        assert accuracy.residual(X, host(Qs[i]), host(Rs[i])) <= 1e-13


def test_batched_fp32_first(scqr, batch_inputs):
    sel = [0, 2, 4, 6, 11, 15]
    Xs = [torch.from_numpy(batch_inputs[i]).cuda() for i in sel]
    Qs, Rs, infos = scqr.qr_batched(Xs, precision="fp32_first")
    for k, i in enumerate(sel):
        X = batch_inputs[i]
        info = infos[k]
        assert info.status == scqr.OK, (i, info)
        ro = oracle.scqr(X, schedule=oracle.ADAPTIVE, precision=1)
        assert info.fell_back_fp64 == ro.fell_back, i
        assert accuracy.orthogonality(host(Qs[k]))[0] <= 1e-13, i
        assert accuracy.residual(X, host(Qs[k]), host(Rs[k])) <= 1e-13, i
        Qs1, Rs1, info1 = scqr.qr(Xs[k], precision="fp32_first")
        assert info1.fell_back_fp64 == info.fell_back_fp64
        if BATCH[i][2] <= 1e10:
            assert info1.passes == info.passes == ro.passes, i


def test_batched_strided_instances(scqr, batch_inputs):
    # per-instance leading dimensions: X_i, Q_i and R_i as column slices of wider buffers give
    # bitwise the contiguous result (the kernels see the same values in the same order)
    sel = [0, 2, 4, 7, 9, 10]
    Xs = [torch.from_numpy(batch_inputs[i]).cuda() for i in sel]
    Qc, Rc, ic = scqr.qr_batched(Xs)
    pads = [3, 1, 8, 5, 2, 9]
    Xw = [torch.full((X.shape[0], X.shape[1] + p), 7.0, dtype=torch.float64, device="cuda") for X, p in zip(Xs, pads)]
    for W, X in zip(Xw, Xs):
        W[:, :X.shape[1]] = X
    Xv = [W[:, :X.shape[1]] for W, X in zip(Xw, Xs)]
    assert all(v.stride(0) > v.shape[1] for v in Xv)
    Q, R, info = scqr.qr_batched(Xv, inplace=True)
    for k in range(len(sel)):
        assert info[k].status == scqr.OK and info[k].passes == ic[k].passes
        assert torch.equal(Xv[k], Qc[k]) and torch.equal(R[k], Rc[k]), k
        assert torch.all(Xw[k][:, Xs[k].shape[1]:] == 7.0)   # the padding columns are untouched


def test_batched_plan_graph_replay(scqr, batch_inputs):
    # the batched plan uploads its descriptors once; run() launches kernels only and is captured
    # in a graph whose replays equal the eager call bitwise, also after new inputs are copied in
    sel = [0, 1, 3, 5, 8, 10, 13]
    shapes = [BATCH[i][:2] for i in sel]
    plan = scqr.BatchedPlan(shapes, "cuda")
    for X, i in zip(plan.Xs, sel):
        X.copy_(torch.from_numpy(batch_inputs[i]))
    plan.run()
    torch.cuda.synchronize()
    Q0 = [q.clone() for q in plan.Qs]
    R0 = [r.clone() for r in plan.Rs]
    i0 = plan.read_infos()
    ref_Q, ref_R, _ = scqr.qr_batched([torch.from_numpy(batch_inputs[i]).cuda() for i in sel])
    for k in range(len(sel)):
        assert i0[k].status == scqr.OK
        assert torch.equal(Q0[k], ref_Q[k]) and torch.equal(R0[k], ref_R[k])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run()   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run()
    for rep in range(3):
        for q in plan.Qs:
            q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(sel)):
            assert torch.equal(plan.Qs[k], Q0[k]) and torch.equal(plan.Rs[k], R0[k]), (rep, k)
        assert [x.passes for x in plan.read_infos()] == [x.passes for x in i0]
    # new values in the captured inputs: the replay factors them
    new = [synth.randsvd(m, n, 1e7, seed=synth.seed_for(4, 500 + j)) for j, (m, n) in enumerate(shapes)]
    for X, A in zip(plan.Xs, new):
        X.copy_(torch.from_numpy(A))
    g.replay()
    torch.cuda.synchronize()
    for k, A in enumerate(new):
        assert plan.read_infos()[k].status == scqr.OK
        assert accuracy.orthogonality(host(plan.Qs[k]))[0] <= 1e-13
        assert accuracy.residual(A, host(plan.Qs[k]), host(plan.Rs[k])) <= 1e-13


def test_batched_tuning_changes_partition_only(scqr, batch_inputs):
    # another row partition (rows per task, 64-row panels) changes only the Gram summation order:
    # same pass counts below kappa 1e12 and the same invariants
    sel = [0, 2, 3, 4, 5, 11, 13, 15]
    Xs = [torch.from_numpy(batch_inputs[i]).cuda() for i in sel]
    tun = {"rows_per_task": [4096, 2048, 8192, 0, 0], "panel_rows": [64, 64, 64, 0, 0]}
    Q1, R1, i1 = scqr.qr_batched(Xs)
    Q2, R2, i2 = scqr.qr_batched(Xs, tuning=tun)
    for k, i in enumerate(sel):
        assert i2[k].status == scqr.OK
        if BATCH[i][2] <= 1e12:
            assert i1[k].passes == i2[k].passes
        X = batch_inputs[i]
        assert accuracy.orthogonality(host(Q2[k]))[0] <= 1e-13, i
        assert accuracy.residual(X, host(Q2[k]), host(R2[k])) <= 1e-13, i
    plan = scqr.BatchedPlan([BATCH[i][:2] for i in sel], "cuda", Xs=Xs, tuning=tun)
    t, nt = plan.tuning_in_effect()
    assert t["panel_rows"][:3] == [64, 64, 64] and t["rows_per_task"][:3] == [4096, 2048, 8192]
    plan.run()
    torch.cuda.synchronize()
    for k in range(len(sel)):
        assert torch.equal(plan.Qs[k], Q2[k]) and torch.equal(plan.Rs[k], R2[k])


def test_batched_argument_errors(scqr):
    X = torch.zeros((100, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        scqr.qr_batched([X], final_gram=True)
    with pytest.raises(Exception):
        scqr.qr_batched([torch.zeros((4, 8), dtype=torch.float64, device="cuda")])


@pytest.mark.slow
@pytest.mark.parametrize("my,n,inst", [((1 << 22) + 37, 64, 11), ((1 << 20) + 37, 256, 12)])
def test_batched_instance_beyond_2_32_elements(scqr, my, n, inst):
    # one batched call holding an instance of about 4.56e9 elements (17 stacked copies of Y,
    # kappa = 1e6) beside two small ones: R = sqrt(17) R_Y and Q = Q_Y / sqrt(17) in every copy
    # against the oracle's factors of Y, and the small instances against the oracle directly
    c = 17
    m = c * my
    assert m * n > 1 << 32 and m < 1 << 31
    sc = np.sqrt(float(c))
    Y = synth.randsvd(my, n, 1e6, seed=synth.seed_for(4, inst))
    smalls = [synth.randsvd(5000, 16, 1e4, seed=synth.seed_for(4, inst + 100)),
              synth.randsvd(3001, 128, 1e6, seed=synth.seed_for(4, inst + 200))]
    Xs = [torch.from_numpy(Y).cuda().repeat(c, 1)] + [torch.from_numpy(S).cuda() for S in smalls]
    print(f"batched call with a {m} x {n} instance ({m * n} elements)", flush=True)
    Qs, Rs, infos = scqr.qr_batched(Xs)
    del Xs
    assert all(i.status == scqr.OK for i in infos)
    ro = oracle.scqr(Y, schedule=oracle.ADAPTIVE)
    Rh = Rs[0].cpu().numpy()
    rerr = np.linalg.norm(Rh - sc * ro.R) / np.linalg.norm(sc * ro.R)
    base = np.concatenate([[0, 1, my - 1], np.random.default_rng(5).choice(my, 61, replace=False)])
    rows = np.concatenate([k * my + base for k in range(c)])
    Qb = Qs[0][torch.from_numpy(rows).cuda()].cpu().numpy().reshape(c, base.size, n)
    qerr = np.max(np.abs(Qb[0] - ro.Q[base] / sc))
    spread = np.max(np.abs(Qb - Qb[0]))
    print(f"passes {infos[0].passes} (oracle on Y {ro.passes}); ||R - sqrt(17) R_Y|| / ||.|| = {rerr:.2e}; "
          f"max |Q - Q_Y / sqrt(17)| = {qerr:.2e}; max spread over copies = {spread:.2e}", flush=True)
    assert rerr <= 1e-10 and qerr <= 1e-10
    assert spread <= 64 * 2.0 ** -53 * np.max(np.abs(Qb[0]))
    assert np.abs(Qb[-1, 2]).max() > 0
    for k, S in enumerate(smalls, start=1):
        rs = oracle.scqr(S, schedule=oracle.ADAPTIVE)
        Rk = Rs[k].cpu().numpy()
        assert np.linalg.norm(Rk - rs.R) <= 1e-10 * np.linalg.norm(rs.R), k
        assert accuracy.orthogonality(Qs[k].cpu().numpy())[0] <= 1e-13, k


def _metrics64(X, Q, R):
    # binary64 BLAS products: their rounding (about sqrt(m) u) stays far below the 1e-13 bar
    n = Q.shape[1]
    om = float(np.max(np.abs(np.linalg.eigvalsh(Q.T @ Q - np.eye(n)))))
    return om, float(np.linalg.norm(X - Q @ R) / np.linalg.norm(X))


@pytest.mark.slow
def test_c4_full_batch_all_instances(scqr):
    """The full 512-instance batch (m_i in [1e4, 2e5], n_i in {16, 32, 64, 128}, kappa_i in
    [1e4, 1e15]) in one batched call, all-FP64 and FP32-first: every instance succeeds with
    ||Q^T Q - I||_2 <= 1e-13 and ||X - QR||_F / ||X||_F <= 1e-13, and the FP32-first R agrees
    with the FP64 R to within kappa_i * 1e-14 (both are backward stable factors of X_i)."""
    spec = synth.batch_spec(512)
    print(f"c4 full batch: generating {len(spec)} instances", flush=True)
    Xh = [synth.randsvd(s.m, s.n, s.kappa, seed=s.seed) for s in spec]
    Xs = [torch.from_numpy(X).cuda() for X in Xh]
    shapes = [(s.m, s.n) for s in spec]
    Rf = None
    for prec in ("fp64", "fp32_first"):
        print(f"c4 full batch: {prec}", flush=True)
        bp = scqr.BatchedPlan(shapes, "cuda", precision=prec)
        bp.run(Xs)
        infos = bp.read_infos()
        Rc = []
        for i, s in enumerate(spec):
            assert infos[i].status == scqr.OK, (prec, i, s, infos[i])
            Qh, Rh = host(bp.Qs[i]), host(bp.Rs[i])
            om, rho = _metrics64(Xh[i], Qh, Rh)
            assert om <= 1e-13 and rho <= 1e-13, (prec, i, s, om, rho)
            assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0), (prec, i)
            Rc.append(Rh)
        if Rf is None:
            Rf = Rc
        else:
            for i, s in enumerate(spec):
                d = np.linalg.norm(Rc[i] - Rf[i]) / np.linalg.norm(Rf[i])
                assert d <= max(s.kappa, 1e2) * 1e-14, (i, s, d)
        del bp
        torch.cuda.empty_cache()


def test_batched_autotune_cached_and_correct(scqr, batch_inputs, tmp_path, monkeypatch):
    """The autotuner times candidate tunings per width class, caches the winner, answers from the
    cache the second time, and a plan built with tuning="auto" factors the batch correctly."""
    import json
    import os

    from paper_1809_11085_amd import autotune

    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("SCQR_AUTOTUNE_CACHE", str(cache))
    sel = [0, 3, 5, 8, 9, 13]
    shapes = [BATCH[i][:2] for i in sel]
    t = autotune.tune(shapes, "cuda", reps=1)
    assert cache.exists()
    stored = json.loads(cache.read_text())
    classes = sorted({scqr.class_of(n) for _, n in shapes})
    assert sorted(v["class"] for v in stored.values()) == classes
    for c in classes:
        sh = [s for s in shapes if scqr.class_of(s[1]) == c]
        assert (t["rows_per_task"][c], t["panel_rows"][c]) in autotune.candidates(c, sh)
    mtime = os.path.getmtime(cache)
    assert autotune.tune(shapes, "cuda", reps=1) == t
    assert os.path.getmtime(cache) == mtime
    Xs = [torch.from_numpy(batch_inputs[i]).cuda() for i in sel]
    plan = scqr.BatchedPlan(shapes, "cuda", Xs=Xs, tuning="auto")
    Qs, Rs = plan.run(Xs)
    infos = plan.read_infos()
    for k, i in enumerate(sel):
        assert infos[k].status == scqr.OK
        Qh, Rh = host(Qs[k]), host(Rs[k])
        assert accuracy.orthogonality(Qh)[0] <= 1e-13
        assert accuracy.residual(batch_inputs[i], Qh, Rh) <= 1e-13
