"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the benchmark.

This module holds no arithmetic of shifted Cholesky QR.  It only draws random numbers and
builds test matrices in the way the paper's numerical experiments describe them:

* ``randsvd``: X = U diag(sigma) V^T with U the orthonormal factor of a Gaussian m x n matrix,
  V the orthonormal factor of a Gaussian n x n matrix and sigma_i = kappa^{-(i-1)/(n-1)}, so
  that ||X||_2 = 1 and kappa_2(X) = kappa (Section 6, equation (testmat), MATLAB's randsvd).
* ``tridiag_b``: a sparse SPD B for the oblique inner product (Section 5) with diagonal
  2 + d_i, d_i log-uniform in [1e-3, 1e3], off-diagonals -1 (stands in for the SuiteSparse
  matrices of Section 7, which are not available).
* ``dense_spd_b``: a dense SPD B = W diag(lambda) W^T with geometric spectrum (Section 6,
  Table 3 construction, B built "as in (testmat)").
* ``stencil_b`` / ``random_pattern_b``: general sparse SPD B in CSR (row pointers, column
  indices, values) with the sparsity of the SuiteSparse matrices of Section 7 (Table of test
  matrices: about 4 to 48 nonzeros per row): a 2-D 5-point or 3-D 27-point stencil pattern, or
  a random symmetric pattern within a band.  Off-diagonal entries are -u_ij, u_ij uniform in
  [0.1, 1] and symmetric; the diagonal is the row's absolute off-diagonal sum plus d_i with
  log10(d_i) uniform in [-3, 3], so B is strictly diagonally dominant, hence SPD.
* ``batch_spec``: shapes and condition numbers for a batch of independent problems.
* ``upstream_grads``: dQ ~ N(0,1), dR = triu(N(0,1)) for the QR adjoint.

The orthonormal factor U of a tall Gaussian matrix is formed block-wise (a two-level
Householder TSQR through ``torch.linalg.qr`` on the CPU, one thread per block) with the
signs normalised so that the triangular factor has a positive diagonal.  Every block draws
from its own ``numpy.random.SeedSequence`` child, so the bytes do not depend on the number of
worker threads.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

BASE_SEED = 180911085
_BLOCK = 16384


def seed_for(config_index: int, instance: int = 0) -> int:
    """Seed of one synthetic problem: base + 1000 * config index + instance."""
    return BASE_SEED + 1000 * int(config_index) + int(instance)


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _householder_q(a: np.ndarray):
    """Orthonormal factor and triangular factor of a (small) matrix via LAPACK Householder QR."""
    import torch

    q, r = torch.linalg.qr(torch.from_numpy(np.ascontiguousarray(a)))
    return q.numpy(), r.numpy()


def _orthonormal_rows_blocks(m: int, n: int, ss: np.random.SeedSequence, block: int, pool):
    """Gaussian m x n drawn block-wise, returned as per-block orthonormal factors Q_b and the
    n x n factor that combines them (two-level TSQR) plus the column-sign vector."""
    nb = (m + block - 1) // block
    kids = ss.spawn(nb)

    def gen_qr(b):
        rows = min(block, m - b * block)
        g = np.random.Generator(np.random.PCG64(kids[b])).standard_normal((rows, n))
        return _householder_q(g)

    res = list(pool.map(gen_qr, range(nb)))
    if nb == 1:
        q, r = res[0]
        return [q], [np.eye(n)], np.sign(np.diag(r))
    stacked = np.vstack([r for _, r in res])
    q2, r2 = _householder_q(stacked)
    return [q for q, _ in res], [q2[b * n:(b + 1) * n] for b in range(nb)], np.sign(np.diag(r2))


def singular_values(n: int, kappa: float) -> np.ndarray:
    """sigma_i = kappa^{-(i-1)/(n-1)}, i = 1..n (sigma_1 = 1, sigma_n = 1/kappa)."""
    if n == 1:
        return np.ones(1)
    e = np.arange(n, dtype=np.float64) / (n - 1)
    return np.power(float(kappa), -e)


def randsvd(m: int, n: int, kappa: float, seed: int, block: int = _BLOCK) -> np.ndarray:
    """X = U diag(sigma) V^T, m x n, float64, C-contiguous (row-major)."""
    import torch

    if m < n or n < 1:
        raise ValueError("randsvd needs m >= n >= 1")
    ss = np.random.SeedSequence(int(seed))
    ss_u, ss_v = ss.spawn(2)
    sigma = singular_values(n, kappa)
    old = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        with ThreadPoolExecutor(_workers()) as pool:
            qs, combs, sgn = _orthonormal_rows_blocks(m, n, ss_u, block, pool)
            gv = np.random.Generator(np.random.PCG64(ss_v)).standard_normal((n, n))
            v, rv = _householder_q(gv)
            v = v * np.sign(np.diag(rv))
            right = (sgn * sigma)[:, None] * v.T  # diag(sign) diag(sigma) V^T
            x = np.empty((m, n), dtype=np.float64)

            def form(b):
                lo = b * block
                x[lo:lo + qs[b].shape[0]] = (qs[b] @ combs[b]) @ right

            list(pool.map(form, range(len(qs))))
    finally:
        torch.set_num_threads(old)
    return x


def gaussian(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) float64 array of the given shape."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed)))).standard_normal(shape)


def tridiag_b(m: int, seed: int):
    """SPD tridiagonal B: diag = 2 + d_i with log10(d_i) ~ U(-3, 3), off-diagonal = -1.

    Returns (diag[m], off[m-1]) as float64 arrays.  B is diagonally dominant with a positive
    diagonal, hence SPD."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 7])))
    d = np.power(10.0, rng.uniform(-3.0, 3.0, size=m))
    return 2.0 + d, -np.ones(max(m - 1, 0))


def dense_spd_b(m: int, kappa_b: float, seed: int) -> np.ndarray:
    """Dense SPD B = W diag(lambda) W^T, W Haar-orthogonal m x m, lambda geometric 1 .. 1/kappa_b."""
    g = gaussian((m, m), seed)
    w, r = np.linalg.qr(g)
    w = w * np.sign(np.diag(r))
    lam = singular_values(m, kappa_b)
    b = (w * lam) @ w.T
    return 0.5 * (b + b.T)


@dataclass(frozen=True)
class CsrB:
    """Symmetric sparse B in compressed sparse row form: row i holds columns
    col[row_ptr[i]:row_ptr[i+1]] (ascending) with values val[...]."""
    row_ptr: np.ndarray  # int64, m + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def m(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        """The m x m matrix (small m only)."""
        b = np.zeros((self.m, self.m))
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        b[rows, self.col] = self.val
        return b


def _spd_from_pairs(m: int, i: np.ndarray, j: np.ndarray, rng) -> CsrB:
    """CSR of the symmetric B with off-diagonal entries (i, j), (j, i) for the given pairs
    (i < j, no repeats): -u_ij, u_ij ~ U(0.1, 1), and a dominant diagonal."""
    u = rng.uniform(0.1, 1.0, size=len(i))
    d = np.power(10.0, rng.uniform(-3.0, 3.0, size=m))
    rows = np.concatenate([i, j, np.arange(m)])
    cols = np.concatenate([j, i, np.arange(m)])
    absum = np.bincount(i, weights=u, minlength=m) + np.bincount(j, weights=u, minlength=m)
    vals = np.concatenate([-u, -u, absum + d])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return CsrB(row_ptr, cols.astype(np.int32), np.ascontiguousarray(vals, dtype=np.float64))


def stencil_b(m: int, kind: str, seed: int) -> CsrB:
    """SPD B in CSR with a finite-difference stencil pattern on a grid of m points numbered
    row by row: '5pt' on a g x ceil(m/g) grid (g = ceil(sqrt m); up to 5 nonzeros per row, like
    apache2, G3_circuit or parabolic_fem), '27pt' on a g x g x ceil(m/g^2) grid (g = ceil(m^(1/3));
    up to 27 per row, like shipsec8 or watercube)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 17])))
    idx = np.arange(m, dtype=np.int64)
    if kind == "5pt":
        g = int(np.ceil(np.sqrt(m)))
        coords = [idx % g, idx // g]
        steps = [(1, 0), (0, 1)]
        strides = [1, g]
    elif kind == "27pt":
        g = int(np.ceil(m ** (1.0 / 3.0)))
        coords = [idx % g, (idx // g) % g, idx // (g * g)]
        steps = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)]
        # half of the neighbours: those with a positive linear offset
        steps = [st for st in steps if st[0] + g * st[1] + g * g * st[2] > 0]
        strides = [1, g, g * g]
    else:
        raise ValueError(kind)
    ii, jj = [], []
    for st in steps:
        off = sum(a * s for a, s in zip(st, strides))
        # a neighbour exists when every coordinate stays on the grid; the last (slowest)
        # coordinate is bounded by the number of points, checked through idx + off < m
        ok = idx + off < m
        for dim, (c, a) in enumerate(zip(coords, st)):
            if a == 1 and dim < len(coords) - 1:
                ok &= c < g - 1
            elif a == -1:
                ok &= c > 0
        ii.append(idx[ok])
        jj.append(idx[ok] + off)
    return _spd_from_pairs(m, np.concatenate(ii), np.concatenate(jj), rng)


def random_pattern_b(m: int, per_row: int, window: int, seed: int) -> CsrB:
    """SPD B in CSR with a random symmetric pattern: row i is coupled to (per_row - 1) / 2 rows
    i + o, o uniform in [1, window] (repeats and pairs past the end dropped), and by symmetry
    to as many below; about per_row nonzeros per row (like bone010, Geo_1438 or serena at 48)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 19])))
    h = max(0, (per_row - 1) // 2)
    i = np.repeat(np.arange(m, dtype=np.int64), h)
    j = i + rng.integers(1, window + 1, size=len(i))
    keep = j < m
    key = np.unique(i[keep] * m + j[keep])
    return _spd_from_pairs(m, key // m, key % m, rng)


@dataclass(frozen=True)
class Instance:
    m: int
    n: int
    kappa: float
    seed: int


def batch_spec(batch: int = 512, config_index: int = 4, m_lo: int = 10000, m_hi: int = 200000,
               ns=(16, 32, 64, 128), log_kappa=(4.0, 15.0)):
    """Per-instance (m_i, n_i, kappa_i, seed_i): m_i uniform integer in [m_lo, m_hi],
    n_i uniform over ``ns``, log10(kappa_i) uniform over ``log_kappa``."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_for(config_index), 11])))
    ms = rng.integers(m_lo, m_hi + 1, size=batch)
    nsel = rng.integers(0, len(ns), size=batch)
    lk = rng.uniform(log_kappa[0], log_kappa[1], size=batch)
    return [Instance(int(ms[i]), int(ns[nsel[i]]), float(10.0 ** lk[i]), seed_for(config_index, i))
            for i in range(batch)]


def upstream_grads(m: int, n: int, seed: int):
    """dQ ~ N(0,1) (m x n) and dR = triu(N(0,1)) (n x n), float64 C-contiguous."""
    ss = np.random.SeedSequence([int(seed), 13])
    a, b = ss.spawn(2)
    dq = np.random.Generator(np.random.PCG64(a)).standard_normal((m, n))
    dr = np.triu(np.random.Generator(np.random.PCG64(b)).standard_normal((n, n)))
    return dq, dr

