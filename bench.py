#!/usr/bin/env python3
"""Benchmark of shifted Cholesky QR on one MI355X.

Default workload: X = U diag(sigma) V^T with m = 2^22, n = 64, sigma geometric from 1 to 1e-15
(kappa ~ 1/u), FP64, Euclidean inner product, the ADAPTIVE schedule (Algorithm 3 followed by
Algorithm 2 continuation) with the paper's shift (eq:finds2).  One step = one complete
factorization X -> (Q, R) with X resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c2|c2b|c1|c3|c5|f1|f3|c4]
                  [--no-extras]

With the default workload the line also carries ``extras``, timed with HIP events on the
launch stream (inputs generated on the host by the seeded generators, then resident in HBM):
  c2b  CholeskyQR2 vs shiftedCholeskyQR3 (Algorithm 3) at kappa = 1e6 (same accuracy bar);
  c3   oblique factorization, 1e6 x 128, kappa = 1e13, tridiagonal SPD B;
  f1   oblique factorization with a sparse SPD B in compressed sparse rows (stencil and random
       banded patterns standing in for the SuiteSparse matrices), 1e6 rows;
  f2   the summation-depth shift against the paper's shift on the default workload;
  f3   minimum-traffic passes (recomputing each pass's input from X) against stored passes;
  c4   512 uneven instances (m_i in [1e4, 2e5], n_i in {16, 32, 64, 128}, kappa_i in
       [1e4, 1e15]): one batched call vs a loop of single calls, and FP32-first vs FP64;
  c5   2^20 x 256, kappa = 1e8: forward (Algorithm 3) and the hand-written adjoint.

The throughput counts the algorithmic flops of the passes actually executed,
passes * (m n (n+1) + m n^2) (one Gram and one triangular solve per pass).  The roofline
object reports the dominant kernel's achieved HBM bandwidth from HIP events recorded on the
launch stream around every kernel of a second, instrumented run of the same K steps; the
cpu_baseline object times the CPU oracle on the same input on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shiftedCholQR3 TFLOP/s & % roofline, m=4M n=64 fp64; mixed/batched speedup"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

WORKLOADS = {
    # name: (m, n, kappa, oblique, description)
    "c2": (1 << 22, 64, 1e15, False, "randsvd m=4194304 n=64 kappa=1e15 fp64, adaptive schedule, paper shift"),
    "c2b": (1 << 22, 64, 1e6, False, "randsvd m=4194304 n=64 kappa=1e6 fp64, adaptive schedule, paper shift"),
    "c1": (4096, 32, 1e12, False, "randsvd m=4096 n=32 kappa=1e12 fp64, adaptive schedule, paper shift"),
    "c3": (1000000, 128, 1e13, True, "randsvd m=1000000 n=128 kappa=1e13, tridiagonal SPD B, fp64"),
    "c5": (1 << 20, 256, 1e8, False, "randsvd m=1048576 n=256 kappa=1e8 fp64, adaptive schedule, paper shift"),
    "f3": (1 << 23, 32, 1e15, False, "randsvd m=8388608 n=32 kappa=1e15 fp64, adaptive schedule, paper shift, "
                                     "minimum-traffic passes"),
    "f1": (1000000, 64, 1e13, True, "randsvd m=1000000 n=64 kappa=1e13, sparse SPD B in compressed sparse rows "
                                    "(3-D 27-point pattern, about 26 entries per row), fp64, adaptive schedule"),
    "c4": (0, 0, 0.0, False, "512 instances m_i in [1e4, 2e5], n_i in {16, 32, 64, 128}, kappa_i in [1e4, 1e15], "
                             "one batched call, fp64"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1809_11085_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def committed_profile(kernel: str, workload: str):
    """The committed rocprofv3 summary of this kernel and workload (profiles/*_counters.json),
    or None when missing or taken from other kernel sources (its source hash differs)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    if c.get("source_hash") != source_hash():
        return None
    return c


def traffic_from_profiles(kernel: str, workload: str, launches_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of this kernel and
    workload, scaled by the copy-kernel calibration, or None when missing or stale."""
    c = committed_profile(kernel, workload)
    return None if c is None else c.get("hbm_bytes_per_launch")


def cpu_baseline(X, passes_gpu, schedule, min_seconds=10.0, max_runs=15):
    """The oracle's complete factorization of the same input, repeated until at least
    min_seconds of wall time have passed; the throughput is the mean over the runs."""
    import oracle

    threads = oracle.num_threads()
    m, n = X.shape
    times = []
    while True:
        t0 = time.perf_counter()
        r = oracle.scqr(X, schedule=schedule)
        times.append(time.perf_counter() - t0)
        if sum(times) >= min_seconds or len(times) >= max_runs:
            break
    dt = sum(times) / len(times)
    flops = r.passes * (m * n * (n + 1) + m * n * n)
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(times)} complete factorizations of the same {m}x{n} input ({r.passes} passes, "
                      f"status {r.status}), {sum(times):.1f} s wall in all, mean {dt:.2f} s each "
                      f"(min {min(times):.2f} s)",
            "seconds": dt, "passes": r.passes}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5):
    """Plain device copies of a known size, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch

    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}))


def peaks():
    """Device ceilings measured with the library's yardstick kernels (scqr_peak_*): streaming
    copy, read and write of 2 GiB (the size of X at m = 2^22, n = 64) over launch widths and
    per-thread unrolls, and the sustained FP64 MFMA 16x16x4 and FP64 FMA rates.  Prints one
    JSON line with the best of each and every measurement."""
    import torch

    import paper_1809_11085_amd as scqr

    torch.cuda.set_device(0)
    nbytes = 1 << 31
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(16384 * 256, dtype=torch.float64, device="cuda")
    rows = []
    for grid in (1024, 2048, 4096):
        for v in range(8):
            ms = _time_ms(lambda: scqr.peak("copy", src, dst, variant=v, grid=grid), reps=5)
            rows.append({"kind": "copy", "grid": grid, "unroll": 1 << (v & 3), "nt_store": bool(v & 4),
                         "GB/s": round(2 * nbytes / ms / 1e6, 1)})
            ms = _time_ms(lambda: scqr.peak("write", dst, variant=v, grid=grid), reps=5)
            rows.append({"kind": "write", "grid": grid, "unroll": 1 << (v & 3), "nt_store": bool(v & 4),
                         "GB/s": round(nbytes / ms / 1e6, 1)})
        for v in range(4):
            ms = _time_ms(lambda: scqr.peak("read", src, sink, variant=v, grid=grid), reps=5)
            rows.append({"kind": "read", "grid": grid, "unroll": 1 << v, "GB/s": round(nbytes / ms / 1e6, 1)})
    iters = 4000
    for grid in (1024, 2048, 4096):
        ms = _time_ms(lambda: scqr.peak("mfma", sink, grid=grid, iters=iters), reps=3)
        fl = grid * 4 * iters * 8 * 2048
        rows.append({"kind": "fp64_mfma_16x16x4", "grid": grid, "TFLOP/s": round(fl / ms / 1e9, 2)})
        ms = _time_ms(lambda: scqr.peak("fma", sink, grid=grid, iters=iters), reps=3)
        fl = grid * 256 * iters * 8 * 2
        rows.append({"kind": "fp64_fma", "grid": grid, "TFLOP/s": round(fl / ms / 1e9, 2)})
    best = {}
    for r in rows:
        key, val = r["kind"], r.get("GB/s", r.get("TFLOP/s"))
        if key not in best or val > best[key]["value"]:
            best[key] = {"value": val, "unit": "GB/s" if "GB/s" in r else "TFLOP/s", "config": r}
    print(json.dumps({"peaks": best, "all": rows, "device": torch.cuda.get_device_name(0)}), flush=True)


def _time_ms(fn, reps=3, warmup=1):
    """Median over reps of the HIP-event time of fn() on the current stream (ms)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def flops_of(m, n, passes):
    return passes * (m * n * (n + 1) + m * n * n)


def extra_c2b(scqr, synth):
    import torch

    m, n = 1 << 22, 64
    X = torch.from_numpy(synth.randsvd(m, n, 1e6, seed=synth.seed_for(1, 2))).cuda()
    out = {}
    for sched in ("fixed3", "cholqr2"):
        plan = scqr.Plan(m, n, "cuda", schedule=sched)
        ms = _time_ms(lambda: plan.run(X), reps=5)
        info = plan.read_info()
        out[sched] = {"ms": round(ms, 4), "passes": info.passes, "status": scqr.status_string(info.status),
                      "TFLOP/s": round(flops_of(m, n, info.passes) / ms / 1e9, 3)}
        del plan
    out["speedup_cholqr2_vs_scholqr3"] = round(out["fixed3"]["ms"] / out["cholqr2"]["ms"], 3)
    del X
    torch.cuda.empty_cache()
    return out


def extra_f2(scqr, synth):
    """c2 (2^22 x 64, kappa = 1e15) with the summation-depth shift: time, passes, the depth the
    library reports and the accuracy, beside the paper's shift, and the oracle's pass count in the
    same mode (its Gram summed in chunks of 2048 rows) beside the oracle's paper-shift count."""
    import numpy as np
    import torch

    import accuracy
    import oracle

    m, n = 1 << 22, 64
    Xh = synth.randsvd(m, n, 1e15, seed=synth.seed_for(1))
    X = torch.from_numpy(Xh).cuda()
    out = {}
    for shift in ("depth", "paper"):
        plan = scqr.Plan(m, n, "cuda", schedule="adaptive", shift=shift)
        ms = _time_ms(lambda: plan.run(X), reps=5)
        info = plan.read_info()
        out[shift] = {"ms": round(ms, 4), "passes": info.passes, "status": scqr.status_string(info.status),
                      "shifts": info.shift, "gram_depth": info.gram_depth,
                      "TFLOP/s": round(flops_of(m, n, info.passes) / ms / 1e9, 3)}
        if shift == "depth":
            Qh, Rh = plan.Q.cpu().numpy(), plan.R.cpu().numpy()
            om, _ = accuracy.orthogonality(Qh)
            out[shift]["orthogonality_2"] = om
            out[shift]["residual"] = accuracy.residual(Xh, Qh, Rh)
        del plan
    chunk = 2048
    rd = oracle.scqr(Xh, schedule=oracle.ADAPTIVE, shift_mode=oracle.SHIFT_DEPTH, gram_chunk=chunk)
    rp = oracle.scqr(Xh, schedule=oracle.ADAPTIVE)
    out["oracle"] = {"depth_mode": {"passes": rd.passes, "status": rd.status, "gram_chunk": chunk,
                                    "gram_depth": oracle.gram_depth(m, chunk), "shifts": rd.shifts},
                     "paper_shift": {"passes": rp.passes, "status": rp.status}}
    out["speedup_depth_vs_paper_shift"] = round(out["paper"]["ms"] / out["depth"]["ms"], 3)
    del X
    torch.cuda.empty_cache()
    return out


def extra_f3(scqr, synth):
    """Minimum-traffic passes (n <= 32): the stored schedule (each pass reads the previous Q and
    writes its own, 8 (2p + 1) m n bytes for p passes) against the recomputing one (passes
    before the last read X and write nothing, 8 (p + 2) m n bytes), on 2^23 rows at n = 32 and
    16, and whether the two give the same factors bit for bit."""
    import torch

    m = 1 << 23
    out = {}
    for n, kappa, sched in ((32, 1e15, "adaptive"), (32, 1e12, "fixed3"), (16, 1e15, "adaptive")):
        X = torch.from_numpy(synth.randsvd(m, n, kappa, seed=synth.seed_for(9, n))).cuda()
        r, fac = {}, {}
        for mt in (False, True):
            key = "recompute" if mt else "stored"
            plan = scqr.Plan(m, n, "cuda", schedule=sched, recompute=mt)
            ms = _time_ms(lambda: plan.run(X), reps=5)
            info = plan.read_info()
            p = info.passes
            nb = 8 * (p + 2) * m * n if mt else 8 * (2 * p + 1) * m * n
            r[key] = {"ms": round(ms, 4), "passes": p, "status": scqr.status_string(info.status),
                      "model_bytes": nb, "GB/s": round(nb / ms / 1e6, 1),
                      "TFLOP/s": round(flops_of(m, n, p) / ms / 1e9, 3)}
            fac[key] = (plan.Q.clone(), plan.R.clone())
            del plan
        r["bitwise_equal"] = bool(torch.equal(fac["stored"][0], fac["recompute"][0]) and
                                  torch.equal(fac["stored"][1], fac["recompute"][1]))
        r["speedup_recompute_vs_stored"] = round(r["stored"]["ms"] / r["recompute"]["ms"], 3)
        out[f"m=2^23 n={n} kappa={kappa:.0e} {sched}"] = r
        del X, fac
        torch.cuda.empty_cache()
    return out


def _csr_dev(scqr, B):
    import torch

    return scqr.CsrB(torch.from_numpy(B.row_ptr).cuda(), torch.from_numpy(B.col).cuda(),
                     torch.from_numpy(B.val).cuda())


def csr_b(synth, kind, m, seed):
    """The sparse SPD B of a CSR workload: '5pt', '27pt' stencil patterns or 'rand' (48 entries per
    row within 4096 rows of the diagonal)."""
    if kind == "rand":
        return synth.random_pattern_b(m, 48, 4096, seed=seed)
    return synth.stencil_b(m, kind, seed=seed)


def extra_f1(scqr, synth):
    """Oblique factorization with a general sparse SPD B in compressed sparse rows (Section 7) on
    stand-ins for the SuiteSparse matrices: 10^6 rows, 5-point (about 5 entries per row, like
    apache2 or G3_circuit), 27-point (about 26, like shipsec8) and random banded (about 47, like
    bone010 or serena) patterns, n = 64, plus n = 16 and 256 on the 27-point pattern; kappa = 1e13,
    adaptive schedule.  Time per factorization, passes, and per kernel the B-Gram against its
    minimum traffic (X, the CSR arrays) and the substitution."""
    import torch

    m = 1000000
    out = {}
    for kind, n in (("5pt", 64), ("27pt", 64), ("rand", 64), ("27pt", 16), ("27pt", 256)):
        B = csr_b(synth, kind, m, seed=synth.seed_for(6, 1))
        X = torch.from_numpy(synth.randsvd(m, n, 1e13, seed=synth.seed_for(6, n))).cuda()
        Bd = _csr_dev(scqr, B)
        plan = scqr.Plan(m, n, "cuda", B=Bd, schedule="adaptive")
        ms = _time_ms(lambda: plan.run(X), reps=5)
        info = plan.read_info()
        scqr.profile_enable(True)
        plan.run(X)
        torch.cuda.synchronize()
        recs = scqr.profile_read()
        scqr.profile_enable(False)
        by = {}
        for name, dur in recs:
            by.setdefault(name, []).append(dur)
        # launches that ran: at least a quarter of the kernel's longest (gated passes return at
        # once, a few microseconds between their events)
        by = {k: [d for d in v if d >= 0.25 * max(v)] for k, v in by.items()}
        p = info.passes
        nnz = B.nnz
        fl = p * (m * n * (n + 1) + m * n * n + 2 * nnz * n) + m * n * (n + 1)
        gb = 8 * m * n + 12 * nnz + 8 * (m + 1)
        r = {"ms": round(ms, 4), "passes": p, "status": scqr.status_string(info.status),
             "nnz_per_row": round(nnz / m, 2), "TFLOP/s": round(fl / ms / 1e9, 3), "bnorm": info.bnorm}
        for k in ("gram_csr_first", "gram_csr", "trsm"):
            if k in by:
                avg = float(sum(by[k]) / len(by[k]))
                r[k] = {"launches": len(by[k]), "avg_ms": round(avg, 4)}
                if k.startswith("gram_csr"):
                    r[k]["GB/s_min_traffic"] = round(gb / avg / 1e6, 1)
                    r[k]["gathered_GB/s"] = round(8 * nnz * n / avg / 1e6, 1)
        out[f"{kind} n={n}"] = r
        del plan, X, Bd, B
        torch.cuda.empty_cache()
    return out


def extra_c3(scqr, synth):
    import torch

    m, n = 1000000, 128
    X = torch.from_numpy(synth.randsvd(m, n, 1e13, seed=synth.seed_for(2))).cuda()
    d, o = synth.tridiag_b(m, seed=synth.seed_for(2, 1))
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    plan = scqr.Plan(m, n, "cuda", B=B, schedule="adaptive")
    ms = _time_ms(lambda: plan.run(X), reps=5)
    info = plan.read_info()
    fl = flops_of(m, n, info.passes) + info.passes * 5 * m * n
    res = {"ms": round(ms, 4), "passes": info.passes, "status": scqr.status_string(info.status),
           "TFLOP/s": round(fl / ms / 1e9, 3), "frac_fp64_peak": round(fl / ms / 1e9 / FP64_PEAK_TFS, 4),
           "shift": info.shift[0], "bnorm": info.bnorm}
    del plan, X
    torch.cuda.empty_cache()
    return res


def _fp64_metrics(X, Q, R):
    """omega_2 = ||Q^T Q - I||_2 and rho = ||X - QR||_F / ||X||_F in plain binary64 (BLAS
    products; their rounding, about sqrt(m) u, stays far below the 1e-13 bar)."""
    import numpy as np

    n = Q.shape[1]
    om = float(np.max(np.abs(np.linalg.eigvalsh(Q.T @ Q - np.eye(n)))))
    rho = float(np.linalg.norm(X - Q @ R) / np.linalg.norm(X))
    return om, rho


def c4_accuracy(scqr, Xs, fp64, mixed, sample_every=16):
    """Per-instance accuracy of the two c4 runs (outside the timed region): omega_2, rho and
    passes for every instance of both runs, the relative R difference between the FP32-first and
    the FP64 run for every instance, and the relative R error of both runs against the CPU
    oracle's FP64 factorization on every sample_every-th instance (about 32 of 512)."""
    import numpy as np

    import oracle

    out = {}
    Rf = []
    Xh_all = [X.cpu().numpy() for X in Xs]
    for name, (Qs, Rs, infos) in (("fp64", fp64), ("fp32_first", mixed)):
        om, rho, rerr = [], [], []
        for i, Xh in enumerate(Xh_all):
            Qh, Rh = Qs[i].cpu().numpy(), Rs[i].cpu().numpy()
            a, b = _fp64_metrics(Xh, Qh, Rh)
            om.append(a)
            rho.append(b)
            if name == "fp64":
                Rf.append(Rh)
            else:
                rerr.append(float(np.linalg.norm(Rh - Rf[i]) / np.linalg.norm(Rf[i])))
        passes = [int(x.passes) for x in infos]
        d = {"omega2_max": max(om), "omega2_median": float(np.median(om)), "rho_max": max(rho),
             "rho_median": float(np.median(rho)), "ok": sum(1 for x in infos if x.status == scqr.OK),
             "within_1e-13": sum(1 for a, b in zip(om, rho) if a <= 1e-13 and b <= 1e-13),
             "passes_hist": {str(k): passes.count(k) for k in sorted(set(passes))}}
        if rerr:
            d["R_rel_diff_vs_fp64_run_max"] = max(rerr)
            d["R_rel_diff_vs_fp64_run_median"] = float(np.median(rerr))
            d["fell_back_fp64"] = sum(1 for x in infos if x.fell_back_fp64)
        out[name] = d
    # against the oracle on a sample covering every width and the whole kappa range
    sample = list(range(0, len(Xs), sample_every))
    err = {"fp64": [], "fp32_first": []}
    kap = []
    for i in sample:
        ro = oracle.scqr(Xh_all[i], schedule=oracle.ADAPTIVE)
        nr = np.linalg.norm(ro.R)
        for name, (Qs, Rs, infos) in (("fp64", fp64), ("fp32_first", mixed)):
            err[name].append(float(np.linalg.norm(Rs[i].cpu().numpy() - ro.R) / nr))
        kap.append(float(np.linalg.cond(ro.R)))
    for name in err:
        e = np.array(err[name])
        out[name]["R_rel_err_vs_oracle_sample"] = {
            "instances": len(sample), "max": float(e.max()), "median": float(np.median(e)),
            "max_over_kappa_u": float(np.max(e / (np.array(kap) * 2.0 ** -53)))}
    return out


def extra_c4(scqr, synth):
    import torch

    spec = synth.batch_spec(512)
    shapes = [(s.m, s.n) for s in spec]
    t0 = time.perf_counter()
    Xs = [torch.from_numpy(synth.randsvd(s.m, s.n, s.kappa, seed=s.seed)).cuda() for s in spec]
    torch.cuda.synchronize()
    log(f"[bench] c4: generated 512 instances in {time.perf_counter() - t0:.1f} s")
    res = {"instances": len(spec), "sum_mn": int(sum(m * n for m, n in shapes))}
    # loop of single calls (each with its own pre-allocated plan)
    plans = [scqr.Plan(m, n, "cuda") for m, n in shapes]

    def loop():
        for pl, X in zip(plans, Xs):
            pl.run(X)

    ms_loop = _time_ms(loop, reps=3)
    passes_loop = [pl.read_info().passes for pl in plans]
    del plans
    torch.cuda.empty_cache()
    bp = scqr.BatchedPlan(shapes, "cuda")
    ms_b = _time_ms(lambda: bp.run(Xs), reps=5)
    infos = bp.read_infos()
    passes = [i.passes for i in infos]
    fl = sum(flops_of(m, n, p) for (m, n), p in zip(shapes, passes))
    res["loop_ms"] = round(ms_loop, 3)
    res["batched_ms"] = round(ms_b, 3)
    res["speedup_batched_vs_loop"] = round(ms_loop / ms_b, 3)
    res["batched_TFLOP/s"] = round(fl / ms_b / 1e9, 3)
    res["ok"] = sum(1 for i in infos if i.status == scqr.OK)
    res["passes_hist"] = {str(k): passes.count(k) for k in sorted(set(passes))}
    res["passes_equal_loop"] = sum(1 for a, b in zip(passes, passes_loop) if a == b)
    bm = scqr.BatchedPlan(shapes, "cuda", precision="fp32_first")
    ms_m = _time_ms(lambda: bm.run(Xs), reps=5)
    im = bm.read_infos()
    res["mixed_batched_ms"] = round(ms_m, 3)
    res["speedup_mixed_vs_fp64_batched"] = round(ms_b / ms_m, 3)
    res["mixed_ok"] = sum(1 for i in im if i.status == scqr.OK)
    res["mixed_fell_back"] = sum(1 for i in im if i.fell_back_fp64)
    t0 = time.perf_counter()
    res["accuracy"] = c4_accuracy(scqr, Xs, (bp.Qs, bp.Rs, infos), (bm.Qs, bm.Rs, im))
    log(f"[bench] c4 accuracy of both runs in {time.perf_counter() - t0:.1f} s")
    del bp, bm, Xs
    torch.cuda.empty_cache()
    return res


def extra_c5(scqr, synth):
    import torch

    m, n = 1 << 20, 256
    X = torch.from_numpy(synth.randsvd(m, n, 1e8, seed=synth.seed_for(5))).cuda()
    dq, dr = synth.upstream_grads(m, n, seed=synth.seed_for(5, 1))
    dQ, dR = torch.from_numpy(dq).cuda(), torch.from_numpy(dr).cuda()
    del dq, dr
    plan = scqr.Plan(m, n, "cuda", schedule="fixed3")
    dX = torch.empty_like(X)
    Q, R = plan.run(X)
    ms_fwd = _time_ms(lambda: plan.run(X), reps=3)
    ms_bwd = _time_ms(lambda: scqr.qr_backward(Q, R, dQ, dR, out=dX), reps=3)
    info = plan.read_info()
    fl_f = flops_of(m, n, info.passes)
    fl_b = 5 * m * n * n
    res = {"forward_ms": round(ms_fwd, 3), "backward_ms": round(ms_bwd, 3), "passes": info.passes,
           "status": scqr.status_string(info.status),
           "forward_TFLOP/s": round(fl_f / ms_fwd / 1e9, 3), "backward_TFLOP/s": round(fl_b / ms_bwd / 1e9, 3),
           "backward_GB/s": round(40 * m * n / ms_bwd / 1e6, 1),
           "backward_over_forward": round(ms_bwd / ms_fwd, 3)}
    del plan, X, dQ, dR, dX, Q, R
    torch.cuda.empty_cache()
    return res


# short names of the single-problem kernels as the library's profiling records them
KERNEL_PATTERNS = [
    # batched: one launch per width class (the class's padded width in the template)
    ("b_trsm_gram_np", r"k_pass_tile<(\d+), 1, false, (true|false), \d+, true>"),
    ("b_gram_np", r"k_pass_tile<(\d+), 0, false, (true|false), \d+, true>"),
    ("b_trsm_gram_np", r"k_pass_wide_b<(\d+)"),
    ("b_gram_np", r"k_gram_wide<(\d+), false, false, false, true>"),
    ("b_chol", r"k_chol_b<"),
    ("b_reduce", r"k_reduce_b\("),
    ("trsm_gram", r"k_pass_tile<\d+, 1, false, (true|false), (32|64)(, false)?>"),
    ("trsm_gram_mt", r"k_pass_tile<\d+, 5, false, (true|false), (32|64)(, false)?>"),
    ("gram", r"k_pass_tile<\d+, 0, (true|false), (true|false), (32|64)(, false)?>"),
    ("trsm", r"k_pass_tile<\d+, 2, false, (true|false), (32|64)(, false)?>"),
    ("gram_csr_first", r"k_gram_csr<\d+, \d+, [123]>"),
    ("gram_csr", r"k_gram_csr<\d+, \d+, 0>"),
    ("trsm_gram", r"k_pass_wide<\d+, 1, (true|false)>"),
    ("trsm", r"k_pass_wide<\d+, 2, (true|false)>"),
    ("trsm_half1", r"k_pass_wide4<"),
    ("gram_b_first", r"k_gram_(wide|lds)<\d+, (\d+, )?true, true"),
    ("gram_b", r"k_gram_(wide|lds)<\d+, (\d+, )?true, false"),
    ("gram", r"k_gram_(wide|lds)<\d+, (\d+, )?false"),
    ("rprod", r"k_mm_breg<"),
    ("chol", r"k_chol<\d+>"),
    ("reduce", r"k_reduce_l[12]\("),
    ("finalize_r", r"k_finalize_r<\d+>"),
]


def alg_bytes(short, m, n, class_mn=None, nnz=None):
    """Algorithmic HBM bytes of one launch: a fused pass or a substitution reads its input and
    writes Q (16 m n; 8 m n for the second half of the n = 256 block solve), a Gram reads its
    input (8 m n; + 16 m for B's two diagonals), the first half of the n = 256 block solve reads
    X and writes Q_1 and X_2' (16 m n); a batched class launch sums 16 m_i n_i or 8 m_i n_i over
    the instances of its width class (class_mn[np] = sum of m_i n_i).  None if not modelled."""
    if short.startswith("b_") and "_np" in short and class_mn is not None:
        np_ = int(short.rsplit("_np", 1)[1])
        per = 16 if short.startswith("b_trsm_gram") else 8
        return per * class_mn.get(np_, 0)
    if short.startswith("gram_csr"):
        # X once, the CSR arrays once (8-byte value, 4-byte column, 8-byte row pointer); the
        # gathered rows of X are re-reads that the caches are expected to serve
        return None if nnz is None else 8 * m * n + 12 * nnz + 8 * (m + 1)
    return {"trsm_gram": 16 * m * n, "trsm": 16 * m * n if n <= 128 else 8 * m * n, "trsm_half1": 16 * m * n,
            "gram": 8 * m * n, "gram_b": 8 * m * n + 16 * m, "gram_b_first": 8 * m * n + 16 * m}.get(short)


def short_name(kname):
    import re

    for short, pat in KERNEL_PATTERNS:
        mt = re.search(pat, kname)
        if mt:
            # batched class kernels carry their padded width: b_trsm_gram_np64, ...
            return short + mt.group(1) if short.endswith("_np") else short
    return None


def summarize_profile(d, workload):
    """Summaries of a rocprofv3 kernel trace and of counter runs of the same bench command:
    FETCH_SIZE and WRITE_SIZE (scaled by what they read for a device copy of known size) and
    FP64 MFMA use, for every kernel of the workload that has a short name.  Writes
    profiles/<kernel>_<workload>.md (text) and _counters.json for the dominant kernel (the
    roofline object of later runs reads its traffic while the kernel sources are unchanged)."""
    import csv

    import numpy as np

    def rows(sub, name):
        with open(os.path.join(d, sub, name)) as fh:
            return list(csv.DictReader(fh))

    m, n = WORKLOADS[workload][:2]
    class_mn = None
    if workload == "c4":
        import synth

        class_mn = {}
        for sp in synth.batch_spec(512):
            np_ = 16
            while np_ < sp.n:
                np_ *= 2
            class_mn[np_] = class_mn.get(np_, 0) + sp.m * sp.n
    nnz = None
    if workload == "f1":
        import synth

        nnz = csr_b(synth, "27pt", m, seed=synth.seed_for(6, 1)).nnz
    trace = rows("trace", "run_kernel_trace.csv")
    stats = rows("trace", "run_kernel_stats.csv")
    per = {}
    for r in trace:
        sn = short_name(r["Kernel_Name"])
        if sn:
            per.setdefault(sn, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    dom = max(per, key=lambda k: sum(per[k]))

    def active(vals, key):
        top = max(key(v) for v in vals)
        return [v for v in vals if key(v) >= 0.25 * top]

    def by_kernel(sub):
        """{short name: {counter: mean over the active dispatches, 'dur': ns}}"""
        out = {}
        disp = {}
        for r in rows(sub, "run_counter_collection.csv"):
            sn = short_name(r["Kernel_Name"])
            if not sn:
                continue
            dd = disp.setdefault((sn, r["Dispatch_Id"]), {"dur": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            dd[r["Counter_Name"]] = float(r["Counter_Value"])
        for (sn, _), v in disp.items():
            out.setdefault(sn, []).append(v)
        res = {}
        for sn, vals in out.items():
            act = active(vals, lambda v: v["dur"])
            res[sn] = {k: float(np.mean([v[k] for v in act])) for k in act[0]}
        return res

    def calib(sub):
        v = [float(r["Counter_Value"]) for r in rows(sub, "run_counter_collection.csv")
             if "copyBuffer" in r["Kernel_Name"]]
        return (1 << 30) / 1024.0 / float(np.median(v))

    fetch, write = by_kernel("fetch"), by_kernel("write")
    util = by_kernel("util") if os.path.isdir(os.path.join(d, "util")) else {}
    fs, ws = calib("cfetch"), calib("cwrite")
    kernels = {}
    for sn, durs in per.items():
        act = active(durs, lambda x: x)
        k = {"launches": len(durs), "active_launches": len(act), "avg_active_ms_rocprof": float(np.mean(act))}
        if sn in fetch and sn in write:
            f, w_ = fetch[sn]["FETCH_SIZE"], write[sn]["WRITE_SIZE"]
            k.update({"fetch_kib_per_launch": f, "write_kib_per_launch": w_,
                      "hbm_bytes_per_launch": f * 1024 * fs + w_ * 1024 * ws})
        alg = alg_bytes(sn, m, n, class_mn, nnz)
        if alg:
            k["algorithmic_bytes_per_launch"] = alg
            k["achieved_GBs"] = alg / (k["avg_active_ms_rocprof"] * 1e-3) / 1e9
            if "hbm_bytes_per_launch" in k:
                k["traffic_over_algorithmic"] = k["hbm_bytes_per_launch"] / alg
        if sn in util:
            u = util[sn]
            cycles = u["GRBM_GUI_ACTIVE"] / 8.0
            k["fp64_mfma"] = {"busy_frac": u["SQ_VALU_MFMA_BUSY_CYCLES"] / (1024.0 * cycles),
                              "tflops": u["SQ_INSTS_VALU_MFMA_F64"] * 2048.0 / (u["dur"] * 1e-9) / 1e12,
                              "clock_ghz": cycles / u["dur"],
                              "lds_bank_conflict_cycles": u.get("SQ_LDS_BANK_CONFLICT")}
        kernels[sn] = k
    base = "python3 -u bench.py --workload %s --steps 5 --warmup 2 --no-cpu-baseline --no-accuracy --no-extras" % workload
    pdir = os.path.relpath(os.path.abspath(d), ROOT)
    short = base.replace("--steps 5 --warmup 2", "--steps 2 --warmup 1")
    rp = "rocprofv3 %s --output-format csv -d " + pdir + "/%s -o run -- %s"
    cmds = {
        "trace": rp % ("--kernel-trace --stats", "trace", base),
        "fetch": rp % ("--kernel-trace --pmc FETCH_SIZE", "fetch", short),
        "write": rp % ("--kernel-trace --pmc WRITE_SIZE", "write", short),
        "util": rp % ("--kernel-trace --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_F64 SQ_LDS_BANK_CONFLICT "
                      "GRBM_GUI_ACTIVE", "util", short),
        "copy_fetch": rp % ("--pmc FETCH_SIZE", "cfetch", "python3 -u bench.py --copy-calibration"),
        "copy_write": rp % ("--pmc WRITE_SIZE", "cwrite", "python3 -u bench.py --copy-calibration"),
        "summary": "python3 bench.py --workload %s --summarize-profile %s" % (workload, pdir),
    }
    kd = kernels[dom]
    out = {"kernel": dom, "workload": workload, "source_hash": source_hash(),
           "avg_active_ms_rocprof": kd["avg_active_ms_rocprof"], "active_launches": kd["active_launches"],
           "hbm_bytes_per_launch": kd.get("hbm_bytes_per_launch"),
           "algorithmic_bytes_per_launch": kd.get("algorithmic_bytes_per_launch"),
           "fetch_scale": fs, "write_scale": ws, "kernels": kernels, "commands": cmds}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{dom}_{workload}_counters.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    lines = [f"# rocprofv3 summary: workload {workload} ({WORKLOADS[workload][4]})", "",
             f"Dominant kernel: `{dom}`.  Commands (run from the repository root on one MI355X):", ""]
    lines += [f"* {k}: `{v}`" for k, v in cmds.items()]
    lines += ["", "## Kernel statistics (`--kernel-trace --stats`, run_kernel_stats.csv)", "",
              "| kernel | calls | total ms | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
        nm = r["Name"].split("(")[0].replace("|", "/")
        lines.append(f"| `{nm[:70]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    lines += ["", "## Per kernel (launches that ran: duration >= 25% of the longest)", "",
              "| kernel | active launches | avg us | alg. bytes | achieved GB/s | HBM traffic / alg. | "
              "FP64 MFMA busy | MFMA TFLOP/s | clock GHz |", "|---|---|---|---|---|---|---|---|---|"]

    def f(v, fmt):
        return "-" if v is None else format(v, fmt)

    for sn, k in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_active_ms_rocprof"] * kv[1]["active_launches"]):
        u = k.get("fp64_mfma") or {}
        lines.append(f"| `{sn}` | {k['active_launches']} | {k['avg_active_ms_rocprof'] * 1e3:.1f} | "
                     f"{f(k.get('algorithmic_bytes_per_launch'), '.4g')} | {f(k.get('achieved_GBs'), '.0f')} | "
                     f"{f(k.get('traffic_over_algorithmic'), '.3f')} | {f(u.get('busy_frac'), '.3f')} | "
                     f"{f(u.get('tflops'), '.1f')} | {f(u.get('clock_ghz'), '.2f')} |")
    if "trsm_gram_mt" in kernels:
        # one kernel for every pass: before the last it reads X and writes nothing (8 m n), the
        # last pass also writes Q (16 m n); listed launch by launch in dispatch order
        def per_dispatch(sub, cname):
            v = {}
            for r in rows(sub, "run_counter_collection.csv"):
                if short_name(r["Kernel_Name"]) == "trsm_gram_mt" and r["Counter_Name"] == cname:
                    v[int(r["Dispatch_Id"])] = (float(r["Counter_Value"]),
                                                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
            return [v[k] for k in sorted(v)]
        fd, wd = per_dispatch("fetch", "FETCH_SIZE"), per_dispatch("write", "WRITE_SIZE")
        seq = [{"read_bytes": fv * 1024 * fs, "written_bytes": wv * 1024 * ws, "ms": fdur}
               for (fv, fdur), (wv, _) in zip(fd, wd)]
        seq = seq[-6:]  # the last factorization: passes 1 .. max_passes = 6 (later ones gated off)
        kernels["trsm_gram_mt"]["per_launch"] = seq
        lines += ["", "## Minimum-traffic passes, launch by launch (`trsm_gram_mt`, counter runs)", "",
                  "The last factorization of each counter run, passes 1 to 6 (a pass after the last one "
                  "returns at once).",
                  f"Model: 8 m n = {8 * m * n:.4g} bytes read per pass; the last pass also writes 8 m n.", "",
                  "| launch | ms (counter run) | HBM read bytes | HBM written bytes | read / 8mn | written / 8mn |",
                  "|---|---|---|---|---|---|"]
        for i, e in enumerate(seq):
            lines.append(f"| {i + 1} | {e['ms']:.3f} | {e['read_bytes']:.4g} | {e['written_bytes']:.4g} | "
                         f"{e['read_bytes'] / (8 * m * n):.3f} | {e['written_bytes'] / (8 * m * n):.3f} |")
    lines += ["", f"A device copy of 1 GiB reads {1048576 / fs:.1f} KiB FETCH_SIZE and {1048576 / ws:.1f} KiB "
              f"WRITE_SIZE, so the counters are scaled by {fs:.4f} and {ws:.4f}.  MFMA busy is "
              "SQ_VALU_MFMA_BUSY_CYCLES over the SIMD-cycles of the launch (1024 SIMDs, GRBM_GUI_ACTIVE / 8 "
              "XCDs cycles); MFMA TFLOP/s counts 2048 flops per FP64 16x16x4 instruction.",
              f"Source hash of the kernels profiled: {out['source_hash']}", ""]
    with open(os.path.join(ROOT, "profiles", f"{dom}_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps({"kernel": dom, "kernels": kernels}))


def run_batched(args, scqr, synth):
    """--workload c4: the 512-instance batch, all FP64, one batched call per step (for profiling
    the per-class launches); one JSON line with the step time and the per-kernel event times."""
    import numpy as np
    import torch

    spec = synth.batch_spec(512)
    shapes = [(s_.m, s_.n) for s_ in spec]
    Xs = [torch.from_numpy(synth.randsvd(s_.m, s_.n, s_.kappa, seed=s_.seed)).cuda() for s_ in spec]
    bp = scqr.BatchedPlan(shapes, "cuda")
    for _ in range(args.warmup):
        bp.run(Xs)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        bp.run(Xs)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    infos = bp.read_infos()
    fl = sum(flops_of(m, n, i.passes) for (m, n), i in zip(shapes, infos))
    scqr.profile_enable(True)
    bp.run(Xs)
    torch.cuda.synchronize()
    recs = scqr.profile_read()
    scqr.profile_enable(False)
    by = {}
    for name, dur in recs:
        by.setdefault(name, []).append(dur)
    print(json.dumps({"workload": WORKLOADS["c4"][4], "ms_per_step": round(ms, 4), "TFLOP/s": round(fl / ms / 1e9, 3),
                      "ok": sum(1 for i in infos if i.status == scqr.OK),
                      "kernels_ms": {k: round(float(np.sum(v)), 4) for k, v in by.items()}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the device ceilings (copy, read, write, FP64 MFMA, FP64 FMA) and exit")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="write profiles/<kernel>_<workload>.md and _counters.json from the rocprofv3 "
                         "outputs under DIR (trace/, fetch/, write/, cfetch/, cwrite/)")
    ap.add_argument("--extras", default="c2b,f1,f2,f3,c3,c4,c5")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the method shards over rows with one n x n "
              "all-reduce per pass, but bench.py runs and reports a single MI355X (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_11085_amd as scqr
    import synth

    if args.copy_calibration:
        copy_calibration()
        return
    if args.peaks:
        peaks()
        return
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.workload)
        return
    if not os.path.exists(scqr.LIB_PATH):
        from paper_1809_11085_amd import build as hipbuild
        hipbuild.build()
    torch.cuda.set_device(0)
    if args.workload == "c4":
        run_batched(args, scqr, synth)
        return
    m, n, kappa, oblique, desc = WORKLOADS[args.workload]
    t = time.perf_counter()
    if args.workload == "f3":
        X = synth.randsvd(m, n, kappa, seed=synth.seed_for(9, n))
    elif args.workload == "f1":
        X = synth.randsvd(m, n, kappa, seed=synth.seed_for(6, n))
    else:
        cfg_index = {"c1": 0, "c2": 1, "c2b": 1, "c3": 2, "c5": 4}[args.workload]
        X = synth.randsvd(m, n, kappa, seed=synth.seed_for(cfg_index))
    B, Bh = None, None
    if args.workload == "f1":
        Bh = csr_b(synth, "27pt", m, seed=synth.seed_for(6, 1))
        B = _csr_dev(scqr, Bh)
    elif oblique:
        d, o = synth.tridiag_b(m, seed=synth.seed_for(cfg_index, 1))
        B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    Xd = torch.from_numpy(X).cuda()
    log(f"[bench] generated {args.workload} {m}x{n} kappa={kappa:.0e} in {time.perf_counter() - t:.1f} s")

    plan = scqr.Plan(m, n, "cuda", B=B, schedule="adaptive", shift="paper", max_passes=6,
                     recompute=args.workload == "f3")
    for _ in range(args.warmup):
        plan.run(Xd)
    torch.cuda.synchronize()
    info = plan.read_info()
    log(f"[bench] warmup done: status={info.status} passes={info.passes} shifts={info.shift}")
    if info.status != scqr.OK:
        log(f"[bench] factorization status {scqr.status_string(info.status)}")

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.run(Xd)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    info = plan.read_info()
    p = info.passes
    flops = p * (m * n * (n + 1) + m * n * n)
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step ({wall:.2f} s wall), {tflops:.2f} TFLOP/s")

    # instrumented run of the same steps: per-kernel durations from events on the launch stream
    scqr.profile_enable(True)
    for _ in range(args.steps):
        plan.run(Xd)
    torch.cuda.synchronize()
    recs = scqr.profile_read()
    scqr.profile_enable(False)
    by = {}
    for name, dur in recs:
        by.setdefault(name, []).append(dur)
    kstats = {}
    for name, ds in by.items():
        top = max(ds)
        active = [d for d in ds if d >= 0.25 * top]
        kstats[name] = {"launches": len(ds), "active_launches": len(active),
                        "avg_active_ms": float(np.mean(active)), "total_ms": float(np.sum(ds))}
    dom = max(kstats, key=lambda k: kstats[k]["total_ms"])
    avg = kstats[dom]["avg_active_ms"]
    # algorithmic bytes per launch of the dominant kernel
    csr_bytes = 8 * m * n + 12 * Bh.nnz + 8 * (m + 1) if Bh is not None else 0
    unit_bytes = {"trsm_gram": 16 * m * n, "trsm": 16 * m * n, "gram": 8 * m * n,
                  "gram_b": 8 * m * n + 16 * m, "gram_b_first": 8 * m * n + 16 * m,
                  "gram_csr": csr_bytes, "gram_csr_first": csr_bytes,
                  # every pass reads X, the last one also writes Q
                  "trsm_gram_mt": 8 * m * n * (p + 1) // max(p, 1)}.get(dom, 16 * m * n)
    achieved = unit_bytes / (avg * 1e-3) / 1e9
    traffic = traffic_from_profiles(dom, args.workload, unit_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": unit_bytes, "avg_launch_ms": round(avg, 5),
                "timing": "HIP events on the launch stream around every launch of this run (primary)"}
    prof = committed_profile(dom, args.workload)
    if prof is not None:
        # the same kernel's average from the committed rocprofv3 kernel trace (same sources)
        a2 = prof["avg_active_ms_rocprof"]
        roofline["avg_launch_ms_rocprof"] = round(a2, 5)
        roofline["frac_rocprof"] = round(unit_bytes / (a2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    # whole-path roofline: bytes (8 + 16 p) m n at 8 TB/s vs flops at 78.6 TFLOP/s; secondary:
    # the minimum-traffic variant that recomputes every Q from X (X read by each pass's Gram and
    # by the final substitution, Q written once: 8 (p + 2) m n bytes, 40 m n at p = 3)
    path_bytes = (8 + 16 * p) * m * n
    t_roof = max(path_bytes / (HBM_PEAK_GBS * 1e9), flops / (FP64_PEAK_TFS * 1e12))
    min_bytes = 8 * (p + 2) * m * n
    result = {
        "metric": METRIC, "value": round(tflops, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "m": m, "n": n, "kappa": kappa, "passes": p,
                   "schedule": "adaptive", "shift": "paper"},
        "roofline": roofline,
        "path_roofline": {"bytes": path_bytes, "flops": flops, "roofline_ms": round(t_roof * 1e3, 4),
                          "frac": round(t_roof * 1e3 / ms, 4),
                          "achieved_GBs": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                          "min_traffic_bytes": min_bytes,
                          "frac_min_traffic": round(min_bytes / (HBM_PEAK_GBS * 1e9) * 1e3 / ms, 4)},
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kstats.items()},
        "status": scqr.status_string(info.status),
    }
    if not args.no_accuracy:
        import accuracy

        t = time.perf_counter()
        Qh, Rh = plan.Q.cpu().numpy(), plan.R.cpu().numpy()
        if Bh is not None:
            om2, omf = accuracy.orthogonality(Qh, csr=(Bh.row_ptr, Bh.col, Bh.val))
        else:
            om2, omf = accuracy.orthogonality(Qh, (d, o) if oblique else None)
        res = accuracy.residual(X, Qh, Rh)
        result["accuracy"] = {"orthogonality_2": om2, "orthogonality_F": omf, "residual": res}
        log(f"[bench] accuracy: ||Q^TQ-I||_2={om2:.2e} residual={res:.2e} ({time.perf_counter() - t:.1f} s)")
    if not args.no_cpu_baseline and not oblique:
        import oracle

        log("[bench] cpu baseline (oracle) ...")
        cb = cpu_baseline(X, p, oracle.ADAPTIVE)
        result["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        result["cpu_baseline"]["value"] = round(cb["value"], 5)
        log(f"[bench] cpu baseline: {cb['value'] * 1e3:.2f} GFLOP/s on {cb['cores']} threads")
    if args.workload == "c2" and not args.no_extras:
        fns = {"c2b": extra_c2b, "f1": extra_f1, "f2": extra_f2, "f3": extra_f3, "c3": extra_c3,
               "c4": extra_c4, "c5": extra_c5}
        extras, speed = {}, {}
        for name in [x for x in args.extras.split(",") if x]:
            t = time.perf_counter()
            try:
                extras[name] = fns[name](scqr, synth)
            except Exception as exc:  # an extra never hides the headline line
                extras[name] = {"error": f"{type(exc).__name__}: {exc}"}
            log(f"[bench] extra {name}: {extras[name]} ({time.perf_counter() - t:.1f} s)")
        for name, key in (("c4", "speedup_batched_vs_loop"), ("c4", "speedup_mixed_vs_fp64_batched"),
                          ("c2b", "speedup_cholqr2_vs_scholqr3"), ("f2", "speedup_depth_vs_paper_shift")):
            if key in extras.get(name, {}):
                speed[f"{name}_{key[8:]}"] = extras[name][key]
        for wl, r in extras.get("f3", {}).items():
            if isinstance(r, dict) and "speedup_recompute_vs_stored" in r:
                speed[f"f3_recompute_vs_stored {wl}"] = r["speedup_recompute_vs_stored"]
        result["speedups"] = speed
        result["extras"] = extras
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
