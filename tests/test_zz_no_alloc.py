"""The no-allocation entry point (scqr_qr_noalloc) against scqr_qr on the same inputs.

The two entry points enqueue the same kernels over the same workspace layout, so their outputs
agree bit for bit.  Two calls in a row, the second on a smaller problem, check that the shared
static scratch carries nothing over from one call to the next."""
import numpy as np
import pytest
import torch

import paper_1809_11085_amd as scqr
import synth

pytestmark = pytest.mark.gpu


def _ref(X, B=None, **opts):
    plan = scqr.Plan(X.shape[0], X.shape[1], X.device, B=B, **opts)
    Q, R = plan.run(X)
    torch.cuda.synchronize()
    return Q.clone(), R.clone(), plan.read_info()


def _noalloc(X, B=None, **opts):
    m, n = X.shape
    Q = torch.full((m, n), float("nan"), dtype=torch.float64, device=X.device)
    R = torch.full((n, n), float("nan"), dtype=torch.float64, device=X.device)
    info = torch.zeros(scqr.INFO_BYTES, dtype=torch.uint8, device=X.device)
    scqr.qr_noalloc(X, Q, R, info, B=B, **opts)
    torch.cuda.synchronize()
    return Q, R, scqr.decode_info(info)


def _same(a, b):
    Qa, Ra, ia = a
    Qb, Rb, ib = b
    assert ia.status == ib.status == scqr.OK
    assert ia.passes == ib.passes and ia.shifted_mask == ib.shifted_mask
    assert ia.shift == ib.shift
    assert torch.equal(Ra, Rb)
    assert torch.equal(Qa, Qb)


def test_noalloc_two_calls_second_smaller():
    cases = [(400_000, 64, 1e15, 1), (5000, 32, 1e12, 2)]
    for m, n, kappa, k in cases:
        print(f"noalloc: m={m} n={n} kappa={kappa:.0e}", flush=True)
        X = torch.from_numpy(synth.randsvd(m, n, kappa, seed=synth.seed_for(0, 90 + k))).cuda()
        got = _noalloc(X)
        _same(got, _ref(X))


def test_noalloc_oblique_and_fixed3_then_smaller():
    m, n = 200_000, 48
    X = torch.from_numpy(synth.randsvd(m, n, 1e10, seed=synth.seed_for(2, 95))).cuda()
    d, o = synth.tridiag_b(m, seed=synth.seed_for(2, 96))
    B = (torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda())
    print(f"noalloc oblique: m={m} n={n}", flush=True)
    _same(_noalloc(X, B=B), _ref(X, B=B))
    X2 = torch.from_numpy(synth.randsvd(3000, 16, 1e8, seed=synth.seed_for(0, 97))).cuda()
    print("noalloc fixed3: m=3000 n=16", flush=True)
    _same(_noalloc(X2, schedule="fixed3"), _ref(X2, schedule="fixed3"))


def test_noalloc_in_place_matches():
    m, n = 100_000, 64
    Xh = synth.randsvd(m, n, 1e9, seed=synth.seed_for(0, 98))
    X = torch.from_numpy(Xh).cuda()
    ref = _ref(X)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    info = torch.zeros(scqr.INFO_BYTES, dtype=torch.uint8, device="cuda")
    scqr.qr_noalloc(X, X, R, info)
    torch.cuda.synchronize()
    _same((X, R, scqr.decode_info(info)), ref)


def test_noalloc_rejects_shapes_beyond_scratch():
    X = torch.zeros((100_000, 128), dtype=torch.float64, device="cuda")
    Q = torch.empty_like(X)
    R = torch.empty((128, 128), dtype=torch.float64, device="cuda")
    info = torch.zeros(scqr.INFO_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(scqr.ScqrError) as ei:
        scqr.qr_noalloc(X, Q, R, info)
    assert ei.value.status == scqr.E_WORKSPACE
    assert not bool(torch.any(info != 0))
