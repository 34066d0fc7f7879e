"""The seeded input generators: exact spectra, determinism, shapes (CPU only)."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("m,n,kappa", [(50, 1, 1.0), (300, 10, 1e8), (40000, 8, 1e12)])
def test_randsvd_spectrum_and_norm(m, n, kappa):
    X = synth.randsvd(m, n, kappa, seed=3)
    assert X.shape == (m, n) and X.dtype == np.float64 and X.flags.c_contiguous
    s = np.linalg.svd(X, compute_uv=False)
    ref = synth.singular_values(n, kappa)
    # singular values are exact up to absolute errors of order u ||X||
    assert np.max(np.abs(s - ref)) < 1e-13
    assert abs(s[0] - 1.0) < 1e-14


def test_randsvd_deterministic_and_seed_dependent():
    a = synth.randsvd(40000, 6, 1e5, seed=9)
    b = synth.randsvd(40000, 6, 1e5, seed=9)
    c = synth.randsvd(40000, 6, 1e5, seed=10)
    np.testing.assert_array_equal(a, b)
    assert np.max(np.abs(a - c)) > 1e-3


def test_randsvd_independent_of_worker_count(monkeypatch):
    a = synth.randsvd(50000, 4, 1e3, seed=12)
    monkeypatch.setattr(synth, "_workers", lambda: 1)
    b = synth.randsvd(50000, 4, 1e3, seed=12)
    np.testing.assert_array_equal(a, b)


def test_singular_values_geometric():
    s = synth.singular_values(5, 1e4)
    np.testing.assert_allclose(s, [1, 1e-1, 1e-2, 1e-3, 1e-4], rtol=1e-14)


def test_tridiag_b_spd_and_range():
    d, o = synth.tridiag_b(2000, seed=1)
    assert d.shape == (2000,) and o.shape == (1999,)
    assert np.all(o == -1.0)
    assert np.all(d >= 2.0 + 1e-3) and np.all(d <= 2.0 + 1e3)
    B = np.diag(d[:300]) + np.diag(o[:299], 1) + np.diag(o[:299], -1)
    assert np.linalg.eigvalsh(B)[0] > 0


def test_dense_spd_b_condition():
    B = synth.dense_spd_b(80, 1e6, seed=2)
    w = np.linalg.eigvalsh(B)
    assert abs(w[-1] - 1.0) < 1e-12 and abs(w[0] * 1e6 - 1) < 1e-4


def test_batch_spec():
    spec = synth.batch_spec(512)
    assert len(spec) == 512
    assert all(10000 <= s.m <= 200000 for s in spec)
    assert {s.n for s in spec} == {16, 32, 64, 128}
    assert all(1e4 <= s.kappa <= 1e15 for s in spec)
    assert len({s.seed for s in spec}) == 512
    assert synth.batch_spec(512) == spec


def test_upstream_grads():
    dq, dr = synth.upstream_grads(100, 7, seed=4)
    assert dq.shape == (100, 7) and dr.shape == (7, 7)
    assert np.all(np.tril(dr, -1) == 0)
    assert abs(np.std(dq) - 1) < 0.1
