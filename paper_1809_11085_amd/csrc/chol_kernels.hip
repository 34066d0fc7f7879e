// Small n x n kernels of shifted Cholesky QR, each run by a single workgroup:
//   * assembly of the Gram from the level-2 partial sums (fixed order),
//   * ||X||_2^2 estimate by power iteration (normest, Section 4.1) or ||X||_F^2,
//   * the shift s of equation (eq:finds2) / (eq:finds2B) (or the FP32-first shift),
//   * R~ = chol(A + sI) with breakdown detection (Algorithm 1 line 3, Algorithm 2 test),
//   * R := R~ R (Algorithms 2 and 3) and the schedule decisions of Algorithms 2, 3, 5,
// all in binary64.  The decisions are written to the device control block and to the
// caller's info record; later kernels of the schedule read them, so the host never waits.
#include "scqr_internal.h"

namespace scqr {

constexpr int kCholThreads = 256;

__device__ double block_sum(double v, double *scratch)
{
    // fixed-order block reduction: lanes by shuffle tree, then waves in order
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// Assemble an np x np symmetric Gram (stride S) from the reduced tiles (gsum, starting at
// element offset `base`); the upper triangle is taken and mirrored, entries beyond n are 0.
// Every thread first issues a chunk of its loads (unrolled) so that they overlap.  The thread's
// share of the checks on the assembled n x n matrix A is accumulated on the way: bad (any entry
// not finite), dev = ||A - I||_F^2 (off-diagonal entries counted twice) and tr = trace(A).
template <int NP>
__device__ __forceinline__ void assemble(const Work &w, int n, int64_t base, bool f32_layout, double *G, int S,
                                         double &bad, double &dev, double &tr)
{
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int CH = T <= 36 ? T : 34;  // all loads in flight at once up to NP = 128, 4 chunks at 256
    // zero the padding only (rows n.., then columns n.. of rows < n); the rest is written below
    const int pad = NP - n;
    for (int idx = threadIdx.x; idx < pad * NP; idx += blockDim.x) G[(n + idx / NP) * S + idx % NP] = 0.0;
    for (int idx = threadIdx.x; idx < n * pad; idx += blockDim.x) G[(idx / pad) * S + n + idx % pad] = 0.0;
    for (int u0 = 0; u0 < T; u0 += CH) {
        double v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (u0 + u < T) v[u] = w.gsum[base + (u0 + u) * 256 + threadIdx.x];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (u0 + u >= T) continue;
            const int e = (u0 + u) * 256 + threadIdx.x;
            int I, J, ii, jj;
            tile_ij(NT, u0 + u, I, J);
            if (f32_layout)
                acc32_rc(e & 255, ii, jj);
            else
                acc64_rc(e & 255, ii, jj);
            const int i = 16 * I + ii, j = 16 * J + jj;
            if (i > j || i >= n || j >= n) continue;
            const double a = v[u];
            G[i * S + j] = a;
            G[j * S + i] = a;
            if (!isfinite(a)) bad = 1.0;
            if (i == j) {
                dev = __builtin_fma(a - 1.0, a - 1.0, dev);
                tr += a;
            } else {
                dev = __builtin_fma(2.0 * a, a, dev);
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void wave_sync_c()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Broadcast lane `src`'s double to every lane (two 32-bit readlanes; src is wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int src)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave, the same value in every lane: within each row of 16 lanes
// by DPP exchanges (quad xor 1, quad xor 2, half-row mirror, row mirror; each lane adds the
// same two operands, so every lane of a row holds the identical row sum), then the four row
// sums ((r0 + r1) + (r2 + r3)).  Fixed order, so the result is deterministic.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Three fixed-order block sums at once: DPP wave sums, then the waves' sums in wave order
// (one pair of barriers for the three).
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *scratch)
{
    a = wave_sum_dpp(a);
    b = wave_sum_dpp(b);
    c = wave_sum_dpp(c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        scratch[3 * wv] = a;
        scratch[3 * wv + 1] = b;
        scratch[3 * wv + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        a += scratch[3 * i];
        b += scratch[3 * i + 1];
        c += scratch[3 * i + 2];
    }
    __syncthreads();
}

// Power iteration of the first wave for NP <= 64 with row i of G held in lane i's registers
// and the iterate broadcast from LDS (the stopping rule and start vector of power_lambda).
template <int NP>
__device__ double power_lambda_regs(const double *G, int S, int n, double *v, const double *v0)
{
    const int lane = threadIdx.x & 63;
    const int row = lane < NP ? lane : NP - 1;
    const bool act = lane < n;
    double g[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) g[k] = (act && k < n) ? G[row * S + k] : 0.0;
    double vi = act ? (v0 ? v0[lane] : 1.0 / sqrt((double)n)) : 0.0;
    if (lane < NP) v[lane] = vi;
    wave_sync_c();
    double lam = 0.0;
    for (int it = 0; it < 100; ++it) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        // the iterate is read from LDS eight entries ahead of its use
        constexpr int CK = NP < 8 ? NP : 8;
        double vb[2][CK];
#pragma unroll
        for (int u = 0; u < CK; ++u) vb[0][u] = v[u];
#pragma unroll
        for (int k0 = 0; k0 < NP; k0 += CK) {
            const int cur = (k0 / CK) & 1;
            if (k0 + CK < NP) {
#pragma unroll
                for (int u = 0; u < CK; ++u) vb[cur ^ 1][u] = v[k0 + CK + u];
            }
#pragma unroll
            for (int u = 0; u < CK; u += 4) {
                a0 = __builtin_fma(g[k0 + u], vb[cur][u], a0);
                a1 = __builtin_fma(g[k0 + u + 1], vb[cur][u + 1], a1);
                a2 = __builtin_fma(g[k0 + u + 2], vb[cur][u + 2], a2);
                a3 = __builtin_fma(g[k0 + u + 3], vb[cur][u + 3], a3);
            }
        }
        const double y = (a0 + a1) + (a2 + a3);
        const double vy = wave_sum_dpp(vi * y);
        const double yy = wave_sum_dpp(y * y);
        const double prev = lam;
        if (!(yy > 0.0)) {
            lam = -1.0;  // G v = 0: the caller falls back to the trace
            break;
        }
        lam = vy;
        const double inv = 1.0 / sqrt(yy);
        vi = y * inv;
        wave_sync_c();
        if (lane < NP) v[lane] = vi;
        wave_sync_c();
        if (it > 0 && fabs(lam - prev) <= 1e-6 * fabs(lam)) break;
    }
    return lam;
}

// Upper Cholesky of G + sI for NP <= 64 by the first wave, right-looking with the trailing
// columns in registers: lane l keeps column l, in blocks of 16 rows whose register positions are
// fixed within a block (the rows shift down by 16 between blocks).  Step j takes the pivot
// radicand from lane j, r_jj = sqrt, r_jl = (entry (j, l)) / r_jj, writes row j of R into G,
// broadcasts it through rb (2 NP doubles, upper half zero) and subtracts r_jk r_jl from every
// remaining entry (k, l).  Each entry therefore receives
// exactly the subtractions a_kl - r_0k r_0l - r_1k r_1l - ... in increasing order followed by
// one division, as in the textbook algorithm.  Entries below the diagonal are not meaningful and
// are never read.  Returns 0 or 1 + the column whose radicand was <= 0 or not finite.
template <int NP>
__device__ __forceinline__ int chol_wave_regs(double *G, int S, int n, double s, double *rb)
{
    static_assert(NP <= 64 && NP % 16 == 0, "one column per lane, 16-row blocks");
    const int l = threadIdx.x & 63;
    const int col = l < NP ? l : NP - 1;
    // block J of 16 steps: c[k] = entry (16 J + k, l); the rows shift down by 16 between blocks
    double c[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double a = G[k * S + col];
        c[k] = (k == l) ? a + s : a;
    }
#pragma unroll
    for (int i = 0; i < 2 * NP; i += 64)
        if (i + l < 2 * NP) rb[i + l] = 0.0;
    wave_sync_c();
    for (int J = 0; 16 * J < n; ++J) {
        const double *rr = rb + 16 * J;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * J + jj;
            if (j >= n) break;
            const double d = readlane_d(c[jj], j);
            if (!(d > 0.0) || !isfinite(d)) return j + 1;
            const double rjj = sqrt(d);
            const double r = (l == j) ? rjj : c[jj] / rjj;
            if (l < NP) {
                G[j * S + l] = r;
                rb[l] = r;
            }
            wave_sync_c();
            // rows below n only: 16-row chunks past n - 1 are skipped
#pragma unroll
            for (int q = 0; q < NP / 16; ++q) {
                if (q > 0 && 16 * J + 16 * q >= n) break;
#pragma unroll
                for (int k = (16 * q > jj + 1 ? 16 * q : jj + 1); k < 16 * q + 16; ++k)
                    c[k] = __builtin_fma(-rr[k], r, c[k]);
            }
            wave_sync_c();
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) c[k] = (k + 16 < NP) ? c[k + 16] : 0.0;
    }
    return 0;
}

// Power iteration for NP = 128 / 256 by the whole workgroup (same start vector, stopping rule and
// iteration cap as power_lambda).  NP = 128: threads 2i and 2i + 1 hold the two halves of
// row i in registers; NP = 256: thread i streams column i (= row i) from G.  The iterate is broadcast from LDS;
// the two sums per iteration are reduced in a fixed order (DPP within each wave, then the four
// wave sums in order), so every thread holds the same values.
template <int NP>
__device__ double power_lambda_block(const double *G, int S, int n, double *v, double *red, const double *v0s)
{
    static_assert(NP == 128 || NP == 256, "block power iteration");
    constexpr int H = NP == 128 ? 2 : 1;       // threads per row
    constexpr int CW = NP / H;                 // columns per thread
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row = t / H, h = t % H;
    const bool act = row < n;
    double g[NP == 128 ? CW : 1];
    if constexpr (NP == 128) {
#pragma unroll
        for (int k = 0; k < CW; ++k) g[k] = (act && CW * h + k < n) ? G[row * S + CW * h + k] : 0.0;
    }
    const double v0 = act ? (v0s ? v0s[row] : 1.0 / sqrt((double)n)) : 0.0;
    __syncthreads();  // v0s may share storage with v
    if (h == 0) v[row] = v0;
    __syncthreads();
    double vi = v0, lam = 0.0;
    for (int it = 0; it < 100; ++it) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if constexpr (NP == 128) {
            const double *vv = v + CW * h;
#pragma unroll
            for (int k = 0; k < CW; k += 4) {
                a0 = __builtin_fma(g[k], vv[k], a0);
                a1 = __builtin_fma(g[k + 1], vv[k + 1], a1);
                a2 = __builtin_fma(g[k + 2], vv[k + 2], a2);
                a3 = __builtin_fma(g[k + 3], vv[k + 3], a3);
            }
        } else {
            // entry (row, k) read as (k, row): G is stored symmetric, and consecutive threads then
            // read consecutive addresses
            const double *gc = G + (act ? row : 0);
            for (int k0 = 0; k0 < NP; k0 += 16) {
                double gb[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) gb[u] = (act && k0 + u < n) ? gc[(k0 + u) * S] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; u += 4) {
                    a0 = __builtin_fma(gb[u], v[k0 + u], a0);
                    a1 = __builtin_fma(gb[u + 1], v[k0 + u + 1], a1);
                    a2 = __builtin_fma(gb[u + 2], v[k0 + u + 2], a2);
                    a3 = __builtin_fma(gb[u + 3], v[k0 + u + 3], a3);
                }
            }
        }
        double y = (a0 + a1) + (a2 + a3);
        if constexpr (H == 2) y = y + dpp_d<0xB1>(y);  // the two halves of the row (quad xor 1)
        const double cvy = (h == 0) ? vi * y : 0.0, cyy = (h == 0) ? y * y : 0.0;
        const double svy = wave_sum_dpp(cvy), syy = wave_sum_dpp(cyy);
        __syncthreads();  // everyone has read v and red
        if (lane == 0) {
            red[2 * wv] = svy;
            red[2 * wv + 1] = syy;
        }
        __syncthreads();
        const double vy = (red[0] + red[2]) + (red[4] + red[6]);
        const double yy = (red[1] + red[3]) + (red[5] + red[7]);
        const double prev = lam;
        if (!(yy > 0.0)) {
            lam = -1.0;  // G v = 0: the caller falls back to the trace
            break;
        }
        lam = vy;
        vi = y * (1.0 / sqrt(yy));
        if (h == 0 && row < NP) v[row] = vi;
        __syncthreads();
        if (it > 0 && fabs(lam - prev) <= 1e-6 * fabs(lam)) break;
    }
    __syncthreads();
    return lam;
}

// ||X||_2^2 estimate (normest's rule: Rayleigh-quotient power iteration on the Gram from the
// start vector 1/sqrt(n), or the unit vector v0 when given, stopped at a relative change <= 1e-6
// or after 100 iterations; a lower bound of lambda_max for any start vector).  NP <= 64: the
// first wave alone, the result broadcast through LDS.  The last iterate is left in v.
// Returns -1 when an iterate falls in the null space of the computed Gram (G v = 0 in
// floating point); the caller then takes the trace instead (||X||_F^2, Section 4.1).
template <int NP>
__device__ __forceinline__ double power_lambda(const double *G, int S, int n, double *v, double *red,
                                               const double *v0 = nullptr)
{
    __syncthreads();
    if constexpr (NP >= 128) {
        return power_lambda_block<NP>(G, S, n, v, red, v0);
    } else {
        if (threadIdx.x < 64) {
            const double lam = power_lambda_regs<NP>(G, S, n, v, v0);
            if (threadIdx.x == 0) red[15] = lam;
        }
        __syncthreads();
        const double lam = red[15];
        __syncthreads();
        return lam;
    }
}


// Blocked right-looking upper Cholesky of G + sI for NP >= 128 by the whole workgroup, in
// 16-column blocks J of the matrix padded to NP with an identity block (rows and columns n..NP-1
// of the upper triangle; the factor of the padded matrix is diag(R, I), so every block is full
// and every loop has compile-time bounds):
//   (1) the 16 x 16 diagonal block is factored by one wave in registers (one column per lane,
//       pivot rows broadcast with readlane);
//   (2) one thread per column solves the block row R_J,K = R_JJ^{-T} A_J,K by forward
//       substitution (multiplying by the reciprocals of the diagonal);
//   (3) the upper tiles of the trailing matrix receive A_KL -= R_J,K^T R_J,L on FP64 MFMA.
// Look-ahead: in (3) the first wave updates the next diagonal tile first and factors it at once
// (step (1) of block J + 1) while the other waves update the remaining tiles, so the diagonal
// factorization is off the critical path.  Every entry is reduced by all earlier rows before its
// own block is factored, as in the textbook algorithm; only the grouping of the subtractions
// differs (by blocks of 16 rows).  Returns 0 or 1 + the first column whose radicand was <= 0 or
// not finite.
template <int NP>
__device__ __forceinline__ int chol_blocked(double *G, int S, int n, double s, double *red, double *dd)
{
    constexpr int NB = NP / 16;
    constexpr int NW = kCholThreads / 64;
    // NP = 256 keeps G in global memory: the current diagonal block and block row are also kept
    // in LDS (block row at the Gram-operand stride), so that steps (2) and (3) read their
    // operands from LDS and only the entries being updated go to global memory
    constexpr bool GG = NP == 256;
    constexpr int BS = lds_stride_gram(NP);
    __shared__ double dbuf[GG ? 256 : 1];
    __shared__ double brow[GG ? 16 * BS : 1];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // entry (i, j) of the current diagonal block and (i, c) of the current block row
    auto rjj_at = [&](int j0, int i, int j) -> double { return GG ? dbuf[i * 16 + j] : G[(j0 + i) * S + j0 + j]; };
    auto brow_at = [&](int j0, int i, int c) -> double { return GG ? brow[i * BS + c] : G[(j0 + i) * S + c]; };
    // (1) for block J by the calling wave: R_JJ into G, its reciprocal diagonal into dd, the
    // breakdown column (or 0) into red[13]
    // (with GG, from_dbuf: the block was just updated into dbuf by this wave)
    auto factor_diag = [&](int J, bool from_dbuf) {
        const int j0 = 16 * J;
        const int col = j0 + li;
        double c[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) c[k] = (GG && from_dbuf) ? dbuf[k * 16 + li] : G[(j0 + k) * S + col];
        int bd = 0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const double d = readlane_d(c[jj], jj);
            if (bd == 0 && (!(d > 0.0) || !isfinite(d))) bd = j0 + jj + 1;
            const double rjj = sqrt(d);
            const double r = (li == jj) ? rjj : c[jj] / rjj;
#pragma unroll
            for (int k = jj + 1; k < 16; ++k) c[k] = __builtin_fma(-readlane_d(r, k), r, c[k]);
            c[jj] = r;
        }
        if (bd == 0 && lane < 16) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k <= lane) G[(j0 + k) * S + j0 + lane] = c[k];
                if (GG) dbuf[k * 16 + lane] = c[k];
                if (k == lane) dd[lane] = 1.0 / c[k];  // reciprocal of r_{j0 + lane, j0 + lane}
            }
        }
        if (lane == 0) red[13] = (double)bd;
    };
    // (3) tile tt of the trailing upper tiles after block J (row-by-row enumeration; tt = 0 is the
    // next diagonal tile)
    auto update_tile = [&](int J, int tt) {
        const int nr = NB - J - 1;
        const int j0 = 16 * J;
        const int K = tile_row(nr, tt), L = tile_col(nr, tt);
        const int k0 = 16 * (J + 1 + K), l0 = 16 * (J + 1 + L);
        d4 d;
#pragma unroll
        for (int r = 0; r < 4; ++r) d[r] = G[(k0 + lk + 4 * r) * S + l0 + li];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int row = 4 * s4 + lk;
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(-brow_at(j0, row, k0 + li), brow_at(j0, row, l0 + li), d, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            G[(k0 + lk + 4 * r) * S + l0 + li] = d[r];
            if (GG && tt == 0) dbuf[(lk + 4 * r) * 16 + li] = d[r];
        }
    };

    for (int idx = t; idx < NP * NP; idx += kCholThreads) {
        const int r = idx / NP, c = idx % NP;
        if (c >= n && r <= c) G[r * S + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int i = t; i < n; i += kCholThreads) G[i * S + i] += s;
    __syncthreads();
    if (wv == 0) factor_diag(0, false);
    __syncthreads();
    for (int J = 0; J < NB; ++J) {
        const int j0 = 16 * J;
        const int bd = (int)red[13];
        if (bd) return bd;
        // (2) block row: r_{j, col} = (a_{j, col} - sum_{i < j} r_{i j} r_{i, col}) / r_jj
        for (int col = j0 + 16 + t; col < NP; col += kCholThreads) {
            double a[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) a[k] = G[(j0 + k) * S + col];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                double v = a[jj];
#pragma unroll
                for (int i = 0; i < jj; ++i) v = __builtin_fma(-rjj_at(j0, i, jj), a[i], v);
                a[jj] = v * dd[jj];
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                G[(j0 + k) * S + col] = a[k];
                if (GG) brow[k * BS + col] = a[k];
            }
        }
        if (J + 1 == NB) break;
        __syncthreads();
        // (3) with look-ahead: the first wave takes the next diagonal tile and factors it, the
        // other waves the remaining tiles
        const int nr = NB - J - 1;
        const int ntile = nr * (nr + 1) / 2;
        if (wv == 0) {
            update_tile(J, 0);
            wave_sync_c();  // the tile's entries were written by other lanes of this wave
            factor_diag(J + 1, true);
        } else if constexpr (GG) {
            // G in global memory: four tiles per round so that their loads overlap
            constexpr int NR = 4;
            for (int t0 = wv; t0 < ntile; t0 += NR * (NW - 1)) {
                d4 d[NR];
                int k0[NR], l0[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const int tt = t0 + q * (NW - 1) < ntile ? t0 + q * (NW - 1) : t0;
                    k0[q] = 16 * (J + 1 + tile_row(nr, tt));
                    l0[q] = 16 * (J + 1 + tile_col(nr, tt));
#pragma unroll
                    for (int r = 0; r < 4; ++r) d[q][r] = G[(k0[q] + lk + 4 * r) * S + l0[q] + li];
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) {
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int row = 4 * s4 + lk;
                        d[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-brow_at(j0, row, k0[q] + li),
                                                                    brow_at(j0, row, l0[q] + li), d[q], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (t0 + q * (NW - 1) >= ntile) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) G[(k0[q] + lk + 4 * r) * S + l0[q] + li] = d[q][r];
                }
            }
        } else {
            for (int tt = wv; tt < ntile; tt += NW - 1) update_tile(J, tt);
        }
        __syncthreads();
    }
    return 0;
}

template <int NP>
__device__ __forceinline__ int chol_inplace(double *G, int S, int n, double s, double *red, double *dd)
{
    if constexpr (NP <= 64) {
        __syncthreads();
        int bd = 0;
        if (threadIdx.x < 64) {
            bd = chol_wave_regs<NP>(G, S, n, s, dd);
            if (threadIdx.x == 0) red[14] = (double)bd;
        }
        __syncthreads();
        bd = (int)red[14];
        __syncthreads();
        return bd;
    }
    __syncthreads();
    return chol_blocked<NP>(G, S, n, s, red, dd);
}

__device__ double shift_value(const SchedParams &sp, int64_t m, int n, double norm2sq,
                              double bfac, bool oblique, bool f32pass, int f32_chain, double sp_depth)
{
    const double dm = (double)m, dn = (double)n;
    if (f32pass)
        return 11.0 * (((double)f32_chain + 2.0) * dn * kU32 + dn * (dn + 1.0) * kU64) * norm2sq;
    double c;
    if (sp.shift_mode == SCQR_SHIFT_DEPTH)
        c = 11.0 * (sp_depth * dn + dn * (dn + 1.0)) * kU64;
    else if (sp.shift_mode == SCQR_SHIFT_SMALL)
        c = kU64;
    else if (sp.shift_mode == SCQR_SHIFT_CUSTOM)
        c = sp.custom_alpha;
    else if (oblique)
        c = 11.0 * (2.0 * dm * sqrt(dm * dn) + dn * (dn + 1.0)) * kU64;
    else
        c = 11.0 * (dm * dn + dn * (dn + 1.0)) * kU64;
    return c * norm2sq * bfac;
}

// variant 0: pass `pass` of the schedule.  variant 1: binary64 redo of pass 1 after the
// FP32-first attempt was rejected.
template <int NP>
__device__ __forceinline__ void chol_body(const Problem &p, const Work &w, const SchedParams &sp, int pass,
                                          int variant)
{
    constexpr bool IN_LDS = NP <= 128;
    constexpr int S = NP + 1;
    __shared__ double lds[IN_LDS ? NP * S : 1];
    __shared__ double vbuf[NP], ybuf[2 * NP], red[16];
    Ctl *ctl = w.ctl;
    scqr_info *info = sp.info;

    {
        const int c_active = ctl->active, c_redo = ctl->redo_fp64, c_pass = ctl->pass, c_last = ctl->last;
        if (variant == 1) {
            if (!(c_active && c_redo)) return;
        } else {
            if (!(c_active && c_pass == pass - 1 && c_last == 0)) return;
        }
    }
    if (ctl->bad_b) {
        // the Gram kernel skipped out-of-range indices of the caller's CSR B
        if (threadIdx.x == 0) {
            ctl->active = 0;
            ctl->status = SCQR_E_INVALID;
            sp.info->status = SCQR_E_INVALID;
            sp.info->passes = pass - 1;
        }
        return;
    }
    const int n = p.n;
    const bool oblique = sp.oblique != 0;
    const bool f32pass = (variant == 0 && pass == 1 && sp.precision == SCQR_PREC_FP32_FIRST);
    const bool obl_first = oblique && pass == 1;
    const int64_t E = (int64_t)upper_tiles(NP / 16) * 256;
    double *G = IN_LDS ? lds : w.G;
    const int bit = 1 << (pass - 1);

    double badd = 0.0, dev = 0.0, tr = 0.0;
    assemble<NP>(w, n, 0, f32pass, G, S, badd, dev, tr);

    // finiteness, ||A - I||_F and trace (the thread shares came with the assembly)
    block_sum3(badd, dev, tr, red);
    const bool bad = badd > 0.0;
    dev = sqrt(dev);
    if (bad && f32pass) {
        // the binary32 Gram overflowed (or X holds a NaN / Inf): redo the first pass in binary64,
        // whose own finiteness test decides the status
        if (threadIdx.x == 0) {
            ctl->redo_fp64 = 1;
            info->fell_back_fp64 = 1;
        }
        return;
    }
    if (bad) {
        if (threadIdx.x == 0) {
            ctl->active = 0;
            ctl->status = SCQR_E_NONFINITE;
            info->status = SCQR_E_NONFINITE;
            info->passes = pass - 1;
        }
        return;
    }
    if (threadIdx.x == 0) {
        info->gram_dev[pass - 1] = dev;
        info->gram_depth = p.gram_depth;
    }
    if (sp.trace) {
        double *tg = sp.trace + (int64_t)(2 * (pass - 1)) * n * n;
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
            const int i = idx / NP, j = idx % NP;
            if (i < n && j < n) tg[i * n + j] = G[i * S + j];
        }
    }

    // norm estimate used by a shift of this pass: the power iteration's lambda_max estimate,
    // raised to max_i a_ii (also a lower bound of lambda_max), or the trace ||.||_F^2 (Section
    // 4.1 allows the Frobenius norm) when the shift mode asks for it or the iteration met G v = 0
    auto norm_estimate = [&]() -> double {
        const double *Gn = G;
        double trn = tr;
        if (obl_first) {
            // ||X||_2 of (eq:finds2B) is the Euclidean norm: Gram X^T X assembled in w.Ge
            double b2 = 0.0, d2 = 0.0, t2 = 0.0;
            assemble<NP>(w, n, E, false, w.Ge, S, b2, d2, t2);
            double t3 = 0.0;
            for (int i = threadIdx.x; i < n; i += blockDim.x) t3 += w.Ge[i * S + i];
            trn = block_sum(t3, red);
            Gn = w.Ge;
        }
        if (sp.shift_mode == SCQR_SHIFT_FRO) return trn;
        // Start vector: after a pass that ran this iteration, R~ v of that pass's last iterate v.
        // Its Gram A' = R~^{-T} A R~^{-1} = I - s (R~ R~^T)^{-1} (with R~^T R~ = A + s I) has the
        // eigenvectors R~ w of A's eigenvectors w, the largest eigenvalue on the largest of A's,
        // so R~ v starts near the dominant eigenvector; the iteration then stops after a few steps
        // where 1/sqrt(n) needs many on the clustered spectrum near 1.  Any start gives a lower
        // bound of lambda_max.
        const double *v0 = nullptr;
        if (!obl_first && pass > 1 && ctl->vprev_pass == pass - 1) {
            const double *Rp = factor_of(w, NP, pass - 1);
            double ss = 0.0;
            for (int i = threadIdx.x; i < NP; i += blockDim.x) {
                double a = 0.0;
                if (i < n)
                    for (int j = i; j < n; ++j) a = __builtin_fma(Rp[i * NP + j], w.vprev[j], a);
                ybuf[i] = a;
                ss += a * a;
            }
            ss = block_sum(ss, red);
            if (ss > 0.0 && isfinite(ss)) {
                const double inv = 1.0 / sqrt(ss);
                for (int i = threadIdx.x; i < NP; i += blockDim.x) ybuf[i] *= inv;
                __syncthreads();
                v0 = ybuf;
            }
        }
        const double lam = power_lambda<NP>(Gn, S, n, vbuf, red, v0);
        if (!(lam >= 0.0)) return trn;
        // keep the last iterate for the next pass's start
        for (int i = threadIdx.x; i < n; i += blockDim.x) w.vprev[i] = vbuf[i];
        if (threadIdx.x == 0) ctl->vprev_pass = pass;
        double dmax = 0.0;
        for (int i = 0; i < n; ++i) dmax = Gn[i * S + i] > dmax ? Gn[i * S + i] : dmax;
        return lam > dmax ? lam : dmax;
    };
    double bfac = 1.0;
    if (obl_first) {
        double b = sp.bnorm_user;
        if (!(b > 0.0)) {
            b = 0.0;
            for (int i = 0; i < w.nwg; ++i) b = w.bmax[i] > b ? w.bmax[i] : b;
        }
        bfac = b;
        if (threadIdx.x == 0) {
            ctl->bnorm = b;
            info->bnorm = b;
        }
    }

    const bool shift_first =
        f32pass || (pass == 1 && (sp.schedule == SCQR_SCHED_FIXED3 || sp.schedule == SCQR_SCHED_ADAPTIVE));
    const bool forced = (sp.force_bd == pass) && variant == 0;
    // First attempt: shifted (Algorithm 3's first pass, FP32-first) or unshifted.  An unshifted
    // attempt that breaks down under the ADAPTIVE / ITERATED schedules is retried once with the
    // shift of this pass (Algorithm 2).  The Cholesky appears once so that it is inlined once.
    const bool may_retry = sp.schedule == SCQR_SCHED_ADAPTIVE || sp.schedule == SCQR_SCHED_ITERATED;
    int shifted = 0, bd = 0;
    double s = 0.0, nrm = 0.0;
    bool try_shift = shift_first;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (try_shift) {
            nrm = norm_estimate();
            s = shift_value(sp, p.m, n, nrm, bfac, oblique, f32pass, f32_chain_rows(NP), p.gram_depth);
            if (sp.zero_shift) s = 0.0;
            shifted = 1;
            if (f32pass && s > 0.01 * nrm) {
                bd = -1;  // binary32 shift too large: redo the first pass in binary64
                break;
            }
        } else {
            s = 0.0;
        }
        bd = (forced && attempt == 0) ? 1 : chol_inplace<NP>(G, S, n, s, red, ybuf);
        if (bd == 0 || try_shift || !may_retry) break;
        if (threadIdx.x == 0) info->breakdown_mask |= bit;
        __syncthreads();
        double b2 = 0.0, d2 = 0.0, t2 = 0.0;
        assemble<NP>(w, n, 0, false, G, S, b2, d2, t2);
        try_shift = true;
    }
    if (f32pass && bd != 0) {
        if (threadIdx.x == 0) {
            ctl->redo_fp64 = 1;
            info->fell_back_fp64 = 1;
        }
        return;
    }
    if (threadIdx.x == 0) {
        info->shift[pass - 1] = s;
        info->norm2sq[pass - 1] = nrm;
        if (shifted) info->shifted_mask |= bit;
    }
    if (bd != 0) {
        if (threadIdx.x == 0) {
            info->breakdown_mask |= bit;
            ctl->active = 0;
            ctl->status = SCQR_E_BREAKDOWN;
            info->status = SCQR_E_BREAKDOWN;
            info->passes = pass - 1;
        }
        return;
    }

    // R~ of this pass (identity padding) and its reciprocal diagonal, in the pass's slot
    double *Rslot = w.Rhist + (int64_t)(pass - 1) * NP * NP;
    double *dslot = w.dhist + (int64_t)(pass - 1) * NP;
#pragma unroll 8
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int i = idx / NP, j = idx % NP;
        double v;
        if (i < n && j < n)
            v = (j >= i) ? G[i * S + j] : 0.0;
        else
            v = (i == j) ? 1.0 : 0.0;
        Rslot[idx] = v;
    }
    for (int i = threadIdx.x; i < NP; i += blockDim.x) dslot[i] = (i < n) ? 1.0 / G[i * S + i] : 1.0;
    if (sp.trace) {
        double *tr_ = sp.trace + (int64_t)(2 * (pass - 1) + 1) * n * n;
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
            const int i = idx / NP, j = idx % NP;
            if (i < n && j < n) tr_[i * n + j] = (j >= i) ? G[i * S + j] : 0.0;
        }
    }

    if (threadIdx.x == 0) {
        int last;
        if (sp.schedule == SCQR_SCHED_FIXED3)
            last = (pass == 3);
        else if (sp.schedule == SCQR_SCHED_CHOLQR2)
            last = (pass == 2);
        else
            last = (!shifted && dev <= 0.5);
        const int maxp = sp.schedule == SCQR_SCHED_FIXED3 ? 3 : sp.schedule == SCQR_SCHED_CHOLQR2 ? 2 : sp.max_passes;
        int status = SCQR_OK;
        if (!last && pass >= maxp) {
            last = 1;
            status = SCQR_E_NOT_CONVERGED;
        }
        ctl->pass = pass;
        ctl->redo_fp64 = 0;
        info->passes = pass;
        if (last) {
            ctl->last = pass;
            ctl->status = status;
            info->status = status;
        }
    }
}

template <int NP>
__global__ void __launch_bounds__(kCholThreads)
k_chol(Problem p, Work w, SchedParams sp, int pass, int variant)
{
    chol_body<NP>(p, w, sp, pass, variant);
}

// Batched form: workgroup i runs the step for instance i (its own info record; no trace).
template <int NP>
__global__ void __launch_bounds__(kCholThreads)
k_chol_b(const BatchInst *__restrict__ insts, SchedParams sp, int pass, int variant)
{
    const BatchInst I = load_cview(insts + blockIdx.x);
    SchedParams spi = sp;
    spi.info = I.info;
    spi.trace = nullptr;
    chol_body<NP>(I.p, I.w, spi, pass, variant);
}

// Initialise the control block and the caller's info record.
__device__ __forceinline__ void init_body(Ctl *ctl, scqr_info *info)
{
    if (threadIdx.x == 0) {
        ctl->active = 1;
        ctl->pass = 0;
        ctl->last = 0;
        ctl->redo_fp64 = 0;
        ctl->status = SCQR_E_NOT_CONVERGED;
        ctl->f32_pass = 0;
        ctl->bad_b = 0;
        ctl->vprev_pass = 0;
        ctl->bnorm = 1.0;
    }
    if (info) {
        int32_t *wi = reinterpret_cast<int32_t *>(info);
        for (int i = threadIdx.x; i < (int)(sizeof(scqr_info) / 4); i += blockDim.x) wi[i] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            info->status = SCQR_E_NOT_CONVERGED;
            info->bnorm = 1.0;
        }
    }
}

__global__ void k_init(Ctl *ctl, scqr_info *info)
{
    init_body(ctl, info);
}

__global__ void k_init_b(const BatchInst *__restrict__ insts)
{
    const BatchInst I = load_cview(insts + blockIdx.x);
    init_body(I.w.ctl, I.info);
}

// G (caller layout, both triangles) from the level-2 partials, for scqr_gram.
template <int NP>
__global__ void __launch_bounds__(256) k_gram_out(Work w, int n, double *G, int64_t ldg)
{
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    const int64_t E = (int64_t)T * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (int64_t)gridDim.x * 256) {
        int I, J, ii, jj;
        tile_ij(NT, (int)(e >> 8), I, J);
        acc64_rc((int)(e & 255), ii, jj);
        const int i = 16 * I + ii, j = 16 * J + jj;
        if (i > j || i >= n || j >= n) continue;
        const double v = w.gsum[e];
        G[(int64_t)i * ldg + j] = v;
        G[(int64_t)j * ldg + i] = v;
    }
}

// Copy a caller's upper triangular R into the padded factor and reciprocal diagonal.
template <int NP>
__global__ void __launch_bounds__(256) k_set_factor(Work w, int n, const double *R, int64_t ldr)
{
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int i = idx / NP, j = idx % NP;
        double v;
        if (i < n && j < n)
            v = (j >= i) ? R[(int64_t)i * ldr + j] : 0.0;
        else
            v = (i == j) ? 1.0 : 0.0;
        w.Rhist[idx] = v;
    }
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w.dhist[i] = (i < n) ? 1.0 / R[(int64_t)i * ldr + i] : 1.0;
}

// R = R~_p ... R~_2 R~_1 over the passes that were applied (R := R~ R of Algorithms 2 and 3),
// written to the caller's R with a zero lower triangle; the identity if no pass was applied.
// One workgroup; the running product stays in LDS when it fits, each entry of a product is a
// sum over k = i..j taken in four interleaved partial sums.
// NP <= 64: thread t owns column j = t % NP of rows g*ROWS .. g*ROWS+ROWS-1 (g = t / NP) of
// each product and accumulates all of them at once over k = 0..NP-1.  Both factors are upper
// triangular with identity padding, so the terms outside i <= k <= j are exact zeros and every
// entry is the k-ordered sum over i..j.  The next factor is loaded while the current product runs.
template <int NP>
__device__ void finalize_small(const Problem &p, const Work &w, int passes)
{
    constexpr int S = NP + 1;       // running product, row-major
    constexpr int ST = NP + 2;      // factor transposed: ft[k * ST + i] = F[i][k]
    constexpr int GR = 256 / NP;    // row groups
    constexpr int ROWS = NP / GR;   // rows per thread
    constexpr int PER = NP * NP / 256;
    __shared__ double A[NP * S];
    __shared__ __attribute__((aligned(16))) double ft[NP * ST];
    const int t = threadIdx.x, j = t % NP, g = t / NP;
    const int n = p.n;

    double nx[PER];
    if (passes >= 1) {
#pragma unroll
        for (int u = 0; u < PER; ++u) nx[u] = w.Rhist[u * 256 + t];
#pragma unroll
        for (int u = 0; u < PER; ++u) A[((u * 256 + t) / NP) * S + (u * 256 + t) % NP] = nx[u];
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = u * 256 + t;
            A[(idx / NP) * S + idx % NP] = (idx / NP == idx % NP) ? 1.0 : 0.0;
        }
    }
    if (passes >= 2) {
#pragma unroll
        for (int u = 0; u < PER; ++u) nx[u] = w.Rhist[(int64_t)NP * NP + u * 256 + t];
    }
    for (int q = 2; q <= passes; ++q) {
        __syncthreads();  // previous product written to A, previous factor no longer read
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = u * 256 + t;
            ft[(idx % NP) * ST + idx / NP] = nx[u];
        }
        if (q < passes) {
            const double *Fn = w.Rhist + (int64_t)q * NP * NP;
#pragma unroll
            for (int u = 0; u < PER; ++u) nx[u] = Fn[u * 256 + t];
        }
        __syncthreads();
        double acc[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
#pragma unroll 4
        for (int k = 0; k < NP; ++k) {
            const double a = A[k * S + j];
            const double *fk = ft + k * ST + g * ROWS;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) acc[r] = __builtin_fma(fk[r], a, acc[r]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ROWS; ++r) A[(g * ROWS + r) * S + j] = acc[r];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = u * 256 + t;
        const int i = idx / NP, jj = idx % NP;
        if (i < n && jj < n) p.R[(int64_t)i * p.ldr + jj] = (jj >= i) ? A[i * S + jj] : 0.0;
    }
}

// NP = 128: the running product in LDS; each factor is staged 16 columns at a time, transposed,
// and thread t accumulates rows 64 (t / 128) .. + 63 of column t % 128 over k in increasing
// order (the terms outside i <= k <= j are exact zeros, as in finalize_small).
template <int NP>
__device__ void finalize_mid(const Problem &p, const Work &w, int passes)
{
    constexpr int S = NP + 1;
    constexpr int KC = 16;
    constexpr int ST = NP + 2;
    constexpr int GR = 256 / NP;
    constexpr int ROWS = NP / GR;
    constexpr int PER = NP * NP / 256;
    constexpr int CH = KC * NP / 256;  // staged values per thread per chunk
    __shared__ double A[NP * S];
    __shared__ __attribute__((aligned(16))) double ft[KC * ST];
    const int t = threadIdx.x, j = t % NP, g = t / NP;
    const int n = p.n;
    for (int u0 = 0; u0 < PER; u0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = (u0 + u) * 256 + t;
            v[u] = passes >= 1 ? w.Rhist[idx] : ((idx / NP == idx % NP) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = (u0 + u) * 256 + t;
            A[(idx / NP) * S + idx % NP] = v[u];
        }
    }
    for (int q = 2; q <= passes; ++q) {
        const double *F = w.Rhist + (int64_t)(q - 1) * NP * NP;
        double acc[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
        for (int k0 = 0; k0 < NP; k0 += KC) {
            double v[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int e = c * 256 + t;
                v[c] = F[(e / KC) * NP + k0 + e % KC];
            }
            __syncthreads();  // the previous chunk (and the previous product) is consumed
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int e = c * 256 + t;
                ft[(e % KC) * ST + e / KC] = v[c];
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < KC; ++kk) {
                const double a = A[(k0 + kk) * S + j];
                const double *fk = ft + kk * ST + g * ROWS;
#pragma unroll
                for (int r = 0; r < ROWS; ++r) acc[r] = __builtin_fma(fk[r], a, acc[r]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ROWS; ++r) A[(g * ROWS + r) * S + j] = acc[r];
    }
    __syncthreads();
    for (int u = 0; u < PER; ++u) {
        const int idx = u * 256 + t;
        const int i = idx / NP, jj = idx % NP;
        if (i < n && jj < n) p.R[(int64_t)i * p.ldr + jj] = (jj >= i) ? A[i * S + jj] : 0.0;
    }
}

// NP = 256: the running product in the global ping-pong buffers.
template <int NP>
__device__ void finalize_big(const Problem &p, const Work &w)
{
    constexpr bool IN_LDS = NP <= 128;
    constexpr int S = NP + 1;
    constexpr int VALS = IN_LDS ? NP * NP / 256 : 1;
    __shared__ double acc_l[IN_LDS ? NP * S : 1];
    __shared__ double fl[NP <= 64 ? NP * NP : 1];
    const int n = p.n;
    const int passes = w.ctl->pass;
    double *A = IN_LDS ? acc_l : w.Racc[0];
    const int sa = IN_LDS ? S : NP;
    if (passes >= 1) {
        // NP*NP/256 loads per thread, all issued before any is used
        constexpr int PER = NP * NP / 256;
        double v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] = w.Rhist[u * 256 + threadIdx.x];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = u * 256 + threadIdx.x;
            A[(idx / NP) * sa + idx % NP] = v[u];
        }
    } else {
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x)
            A[(idx / NP) * sa + idx % NP] = ((idx / NP) == (idx % NP)) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int q = 2; q <= passes; ++q) {
        const double *F = w.Rhist + (int64_t)(q - 1) * NP * NP;
        if (NP <= 64) {  // stage the factor in LDS next to the running product
            constexpr int PER = NP * NP / 256;
            double v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) v[u] = F[u * 256 + threadIdx.x];
#pragma unroll
            for (int u = 0; u < PER; ++u) fl[u * 256 + threadIdx.x] = v[u];
            __syncthreads();
            F = fl;
        }
        double *D = IN_LDS ? nullptr : w.Racc[(q & 1) ? 0 : 1];  // global ping-pong target
        const double *Asrc = A;
        double vals[VALS];
        int cnt = 0;
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x, ++cnt) {
            const int i = idx / NP, j = idx % NP;
            double v = 0.0;
            if (j >= i && i < n && j < n) {
                // new[i][j] = sum_{k=i..j} F[i][k] A[k][j], four interleaved partial sums
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int k = i;
                for (; k + 4 <= j + 1; k += 4) {
                    a0 = __builtin_fma(F[i * NP + k], Asrc[k * sa + j], a0);
                    a1 = __builtin_fma(F[i * NP + k + 1], Asrc[(k + 1) * sa + j], a1);
                    a2 = __builtin_fma(F[i * NP + k + 2], Asrc[(k + 2) * sa + j], a2);
                    a3 = __builtin_fma(F[i * NP + k + 3], Asrc[(k + 3) * sa + j], a3);
                }
                for (; k <= j; ++k) a0 = __builtin_fma(F[i * NP + k], Asrc[k * sa + j], a0);
                v = (a0 + a1) + (a2 + a3);
            } else if (i >= n || j >= n) {
                v = (i == j) ? 1.0 : 0.0;
            }
            if (IN_LDS)
                vals[cnt < VALS ? cnt : 0] = v;
            else
                D[idx] = v;
        }
        __syncthreads();
        if (IN_LDS) {
            cnt = 0;
            for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x, ++cnt)
                A[(idx / NP) * sa + idx % NP] = vals[cnt < VALS ? cnt : 0];
        } else {
            A = D;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int i = idx / NP, j = idx % NP;
        if (i < n && j < n) p.R[(int64_t)i * p.ldr + j] = (j >= i) ? A[i * sa + j] : 0.0;
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_finalize_r(Problem p, Work w)
{
    if constexpr (NP <= 64)
        finalize_small<NP>(p, w, w.ctl->pass);
    else if constexpr (NP == 128)
        finalize_mid<NP>(p, w, w.ctl->pass);
    else
        finalize_big<NP>(p, w);
}

// NP = 128 / 256 after launch_rprod: R from P_passes (the identity when no pass was applied).
template <int NP>
__global__ void __launch_bounds__(256) k_finalize_copy(Problem p, Work w)
{
    const int passes = w.ctl->pass;
    const double *src = passes >= 2 ? w.Racc[passes & 1] : w.Rhist;
    const int n = p.n;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n * n; e += gridDim.x * 256) {
        const int i = e / n, j = e % n;
        double v = 0.0;
        if (j >= i) v = passes >= 1 ? src[i * NP + j] : (i == j ? 1.0 : 0.0);
        p.R[(int64_t)i * p.ldr + j] = v;
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_finalize_b(const BatchInst *__restrict__ insts)
{
    const BatchInst I = load_cview(insts + blockIdx.x);
    if constexpr (NP <= 64)
        finalize_small<NP>(I.p, I.w, I.w.ctl->pass);
    else if constexpr (NP == 128)
        finalize_mid<NP>(I.p, I.w, I.w.ctl->pass);
    else
        finalize_big<NP>(I.p, I.w);
}

// ||G - I||_F of the final Gram (final_gram option).
template <int NP>
__global__ void __launch_bounds__(256) k_final_omega(Problem p, Work w, SchedParams sp)
{
    __shared__ double red[16];
    Ctl *ctl = w.ctl;
    if (!(ctl->active && ctl->last > 0)) return;
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    const int n = p.n;
    double acc = 0.0;
    for (int e = threadIdx.x; e < T * 256; e += blockDim.x) {
        int I, J, ii, jj;
        tile_ij(NT, e >> 8, I, J);
        acc64_rc(e & 255, ii, jj);
        const int i = 16 * I + ii, j = 16 * J + jj;
        if (i > j || i >= n || j >= n) continue;
        const double d = w.gsum[e] - (i == j ? 1.0 : 0.0);
        acc += (i == j ? 1.0 : 2.0) * d * d;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) sp.info->omega_fro = sqrt(acc);
}

// ------------------------------------------------------------------------------------------
hipError_t launch_chol(hipStream_t s, const Problem &p, const Work &w, const SchedParams &sp,
                       int pass, int variant)
{
    prof_before(s, "chol");
    switch (p.np) {
    case 16: hipLaunchKernelGGL((k_chol<16>), dim3(1), dim3(kCholThreads), 0, s, p, w, sp, pass, variant); break;
    case 32: hipLaunchKernelGGL((k_chol<32>), dim3(1), dim3(kCholThreads), 0, s, p, w, sp, pass, variant); break;
    case 64: hipLaunchKernelGGL((k_chol<64>), dim3(1), dim3(kCholThreads), 0, s, p, w, sp, pass, variant); break;
    case 128: hipLaunchKernelGGL((k_chol<128>), dim3(1), dim3(kCholThreads), 0, s, p, w, sp, pass, variant); break;
    case 256: hipLaunchKernelGGL((k_chol<256>), dim3(1), dim3(kCholThreads), 0, s, p, w, sp, pass, variant); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t s, const Problem &, const Work &w, const SchedParams &sp)
{
    prof_before(s, "init");
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, w.ctl, sp.info);
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_gram_out(hipStream_t s, const Work &w, int np, int n, double *G, int64_t ldg)
{
    prof_before(s, "gram_out");
    switch (np) {
    case 16: hipLaunchKernelGGL((k_gram_out<16>), dim3(4), dim3(256), 0, s, w, n, G, ldg); break;
    case 32: hipLaunchKernelGGL((k_gram_out<32>), dim3(4), dim3(256), 0, s, w, n, G, ldg); break;
    case 64: hipLaunchKernelGGL((k_gram_out<64>), dim3(16), dim3(256), 0, s, w, n, G, ldg); break;
    case 128: hipLaunchKernelGGL((k_gram_out<128>), dim3(64), dim3(256), 0, s, w, n, G, ldg); break;
    case 256: hipLaunchKernelGGL((k_gram_out<256>), dim3(128), dim3(256), 0, s, w, n, G, ldg); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_set_factor(hipStream_t s, const Work &w, int np, int n, const double *R, int64_t ldr)
{
    prof_before(s, "set_factor");
    switch (np) {
    case 16: hipLaunchKernelGGL((k_set_factor<16>), dim3(1), dim3(256), 0, s, w, n, R, ldr); break;
    case 32: hipLaunchKernelGGL((k_set_factor<32>), dim3(1), dim3(256), 0, s, w, n, R, ldr); break;
    case 64: hipLaunchKernelGGL((k_set_factor<64>), dim3(1), dim3(256), 0, s, w, n, R, ldr); break;
    case 128: hipLaunchKernelGGL((k_set_factor<128>), dim3(1), dim3(256), 0, s, w, n, R, ldr); break;
    case 256: hipLaunchKernelGGL((k_set_factor<256>), dim3(1), dim3(256), 0, s, w, n, R, ldr); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_finalize_r(hipStream_t s, const Problem &p, const Work &w, int maxp)
{
    if (p.np >= 128) {
        prof_before(s, "finalize_r");
        hipError_t e = launch_rprod(s, w, p.np, maxp);
        if (e == hipSuccess) {
            if (p.np == 256)
                hipLaunchKernelGGL((k_finalize_copy<256>), dim3(64), dim3(256), 0, s, p, w);
            else
                hipLaunchKernelGGL((k_finalize_copy<128>), dim3(64), dim3(256), 0, s, p, w);
        }
        prof_after(s);
        return e == hipSuccess ? hipGetLastError() : e;
    }
    prof_before(s, "finalize_r");
    switch (p.np) {
    case 16: hipLaunchKernelGGL((k_finalize_r<16>), dim3(1), dim3(256), 0, s, p, w); break;
    case 32: hipLaunchKernelGGL((k_finalize_r<32>), dim3(1), dim3(256), 0, s, p, w); break;
    case 64: hipLaunchKernelGGL((k_finalize_r<64>), dim3(1), dim3(256), 0, s, p, w); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_final_omega(hipStream_t s, const Problem &p, const Work &w, const SchedParams &sp)
{
    prof_before(s, "final_omega");
    switch (p.np) {
    case 16: hipLaunchKernelGGL((k_final_omega<16>), dim3(1), dim3(256), 0, s, p, w, sp); break;
    case 32: hipLaunchKernelGGL((k_final_omega<32>), dim3(1), dim3(256), 0, s, p, w, sp); break;
    case 64: hipLaunchKernelGGL((k_final_omega<64>), dim3(1), dim3(256), 0, s, p, w, sp); break;
    case 128: hipLaunchKernelGGL((k_final_omega<128>), dim3(1), dim3(256), 0, s, p, w, sp); break;
    case 256: hipLaunchKernelGGL((k_final_omega<256>), dim3(1), dim3(256), 0, s, p, w, sp); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

// ---- batched launchers (one workgroup per instance) ----------------------------------------
hipError_t launch_init_b(hipStream_t s, const BatchClass &c)
{
    if (c.ninst <= 0) return hipSuccess;
    prof_before(s, "b_init");
    hipLaunchKernelGGL(k_init_b, dim3((unsigned)c.ninst), dim3(256), 0, s, c.insts);
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_chol_b(hipStream_t s, const BatchClass &c, const SchedParams &sp, int pass, int variant)
{
    if (c.ninst <= 0) return hipSuccess;
    dim3 grid((unsigned)c.ninst), block(kCholThreads);
    prof_before(s, "b_chol");
    switch (c.np) {
    case 16: hipLaunchKernelGGL((k_chol_b<16>), grid, block, 0, s, c.insts, sp, pass, variant); break;
    case 32: hipLaunchKernelGGL((k_chol_b<32>), grid, block, 0, s, c.insts, sp, pass, variant); break;
    case 64: hipLaunchKernelGGL((k_chol_b<64>), grid, block, 0, s, c.insts, sp, pass, variant); break;
    case 128: hipLaunchKernelGGL((k_chol_b<128>), grid, block, 0, s, c.insts, sp, pass, variant); break;
    case 256: hipLaunchKernelGGL((k_chol_b<256>), grid, block, 0, s, c.insts, sp, pass, variant); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_finalize_b(hipStream_t s, const BatchClass &c)
{
    if (c.ninst <= 0) return hipSuccess;
    dim3 grid((unsigned)c.ninst), block(256);
    prof_before(s, "b_finalize_r");
    switch (c.np) {
    case 16: hipLaunchKernelGGL((k_finalize_b<16>), grid, block, 0, s, c.insts); break;
    case 32: hipLaunchKernelGGL((k_finalize_b<32>), grid, block, 0, s, c.insts); break;
    case 64: hipLaunchKernelGGL((k_finalize_b<64>), grid, block, 0, s, c.insts); break;
    case 128: hipLaunchKernelGGL((k_finalize_b<128>), grid, block, 0, s, c.insts); break;
    case 256: hipLaunchKernelGGL((k_finalize_b<256>), grid, block, 0, s, c.insts); break;
    default: prof_after(s); return hipErrorInvalidValue;
    }
    prof_after(s);
    return hipGetLastError();
}

}  // namespace scqr
