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


def _grid_neighbours(kind, m, i):
    """Neighbours of grid point i written out from the stencil's definition."""
    if kind == "5pt":
        g = int(np.ceil(np.sqrt(m)))
        return {j for j in (i - 1, i + 1, i - g, i + g) if 0 <= j < m and (abs(j - i) != 1 or j // g == i // g)}
    g = int(np.ceil(m ** (1.0 / 3.0)))
    x, y, z = i % g, (i // g) % g, i // (g * g)
    out = set()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                X, Y, Z = x + dx, y + dy, z + dz
                if (dx, dy, dz) != (0, 0, 0) and 0 <= X < g and 0 <= Y < g and Z >= 0 and X + g * Y + g * g * Z < m:
                    out.add(X + g * Y + g * g * Z)
    return out


@pytest.mark.parametrize("kind,m", [("5pt", 37), ("5pt", 1000), ("27pt", 37), ("27pt", 1000)])
def test_stencil_b_pattern_and_spd(kind, m):
    B = synth.stencil_b(m, kind, seed=5)
    assert B.row_ptr.dtype == np.int64 and B.col.dtype == np.int32 and B.val.dtype == np.float64
    assert B.row_ptr[0] == 0 and B.nnz == len(B.col) == len(B.val)
    for i in range(m):
        cols = B.col[B.row_ptr[i]:B.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)  # ascending, no repeats
        assert set(cols.tolist()) - {i} == _grid_neighbours(kind, m, i)
    D = B.dense()
    np.testing.assert_array_equal(D, D.T)
    off = D - np.diag(np.diag(D))
    assert np.all(np.diag(D) - np.abs(off).sum(axis=1) >= 1e-3 * (1 - 1e-12))  # dominant diagonal
    assert np.linalg.eigvalsh(D)[0] > 0
    assert synth.stencil_b(m, kind, seed=5).val.tobytes() == B.val.tobytes()


def test_random_pattern_b():
    m = 3000
    B = synth.random_pattern_b(m, 48, 200, seed=6)
    D = B.dense()
    np.testing.assert_array_equal(D, D.T)
    assert np.linalg.eigvalsh(D)[0] > 0
    rows = np.repeat(np.arange(m), np.diff(B.row_ptr))
    assert np.all(np.abs(B.col - rows) <= 200)
    assert 40 <= B.nnz / m <= 48
    for i in range(0, m, 97):
        assert np.all(np.diff(B.col[B.row_ptr[i]:B.row_ptr[i + 1]]) > 0)
