"""Autotuner of the batched schedule: rows per task and panel rows per width class.

A batched call groups its instances into width classes (padded n = 16, 32, 64, 128, 256) and
cuts each class's rows into tasks, one workgroup each.  How many rows a task takes trades the
tail of a launch (few large tasks leave compute units idle at the end) against per-task
overhead (many small tasks repeat the factor staging and write more partial Grams).  The best
split depends on the batch and the device, so it is measured: for every class present, each
candidate tuning is timed on a batch holding only that class's shapes (classes run in separate
launches, so their tunings are independent), and the fastest is kept.

Results are cached in a JSON file keyed by the device, the library build, the options that
change the schedule, and the shapes of each class (``SCQR_AUTOTUNE_CACHE`` overrides the file;
default ``~/.cache/scqr/autotune.json``).  The timed inputs are random normal matrices of the
same shapes; timing does not depend on the values except through the pass count, which the
FIXED3 schedule used for the trials keeps at three.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

ROWS_CANDIDATES = (1024, 2048, 4096, 8192, 16384)
PANEL_CANDIDATES = (32, 64)


def cache_path() -> str:
    p = os.environ.get("SCQR_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "scqr", "autotune.json")


def _load_cache(path):
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def class_key(device, shapes, precision) -> str:
    """Cache key of one class: device, library build, precision and the sorted shapes."""
    from . import build_info

    props = torch.cuda.get_device_properties(device)
    h = hashlib.sha256()
    h.update(f"{props.name}|{props.multi_processor_count}|{build_info()}|{precision}|".encode())
    h.update(json.dumps(sorted(shapes)).encode())
    return h.hexdigest()[:24]


def _time_plan(plan, Xs, reps):
    plan.run(Xs)  # warm-up (and binding)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        plan.run(Xs)
        b.record(st)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def candidates(c: int, shapes):
    """Candidate (rows_per_task, panel_rows) of class c for these shapes; rows_per_task 0 is the
    library default, panel_rows 0 the library default (32)."""
    mmax = max(m for m, _ in shapes)
    rows = [0] + [r for r in ROWS_CANDIDATES if r < 2 * mmax]
    panels = PANEL_CANDIDATES if c <= 2 else (0,)
    return [(r, p) for r in rows for p in panels]


def tune(shapes, device="cuda", reps=3, precision="fp64", verbose=False, **opts):
    """Tuning dict {"rows_per_task": [5], "panel_rows": [5]} for a batch of (m, n) shapes,
    measured on `device` (or read from the cache)."""
    from . import BatchedPlan, class_of, NUM_CLASSES

    dev = torch.device(device)
    opts = {k: v for k, v in opts.items() if k not in ("schedule", "max_passes")}
    path = cache_path()
    cache = _load_cache(path)
    by = {}
    for m, n in shapes:
        by.setdefault(class_of(int(n)), []).append((int(m), int(n)))
    out = {"rows_per_task": [0] * NUM_CLASSES, "panel_rows": [0] * NUM_CLASSES}
    changed = False
    for c, sh in sorted(by.items()):
        key = class_key(dev, sh, precision)
        if key in cache:
            rpt, pr = cache[key]["rows_per_task"], cache[key]["panel_rows"]
        else:
            gen = torch.Generator(device=dev).manual_seed(1809)
            Xs = [torch.randn((m, n), dtype=torch.float64, device=dev, generator=gen) for m, n in sh]
            trials = []
            for rpt, pr in candidates(c, sh):
                t = {"rows_per_task": [0] * NUM_CLASSES, "panel_rows": [0] * NUM_CLASSES}
                t["rows_per_task"][c], t["panel_rows"][c] = rpt, pr
                plan = BatchedPlan(sh, dev, Xs=Xs, tuning=t, schedule="fixed3", precision=precision, **opts)
                trials.append((_time_plan(plan, Xs, reps), rpt, pr))
                del plan
            trials.sort()
            _, rpt, pr = trials[0]
            cache[key] = {"rows_per_task": rpt, "panel_rows": pr, "class": c, "instances": len(sh),
                          "trials_ms": [[round(ms, 4), r, p] for ms, r, p in trials]}
            changed = True
            if verbose:
                print(f"autotune class {c}: {len(sh)} instances, best rows_per_task={rpt} "
                      f"panel_rows={pr} ({trials[0][0]:.3f} ms of {len(trials)} trials)", flush=True)
            del Xs
        out["rows_per_task"][c], out["panel_rows"][c] = rpt, pr
    if changed:
        _store_cache(path, cache)
    return out
