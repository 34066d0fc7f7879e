// QR adjoint on gfx950 (reverse-mode derivative of X -> (Q, R), thin QR with positive diag):
//   G = dQ^T Q (split-m, FP64 MFMA, fixed-order reduction),
//   M = R dR^T - G,  C = copyltu(M)  (C_ij = M_{max(i,j), min(i,j)}),
//   dX = (dQ + Q C) R^{-T}, row by row: y^T = dq^T + q^T C, then dx^T R^T = y^T by back
//   substitution (column sweep from the last column).
#include "scqr_internal.h"

namespace scqr {

namespace {

struct BwdWork {
    double *partials;  // nwg x NT^2 * 256
    double *lvl2;      // nlvl2 x NT^2 * 256
    double *C;         // np x np
    double *RT;        // np x np, RT[k][i] = R[i][k] (identity padding)
    double *dinv;      // np
    int nwg, nlvl2;
};

int bwd_grid(int64_t m)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t panels = (m + 15) / 16;
    const int64_t cap = 2 * (int64_t)(cus > 0 ? cus : 256);
    const int64_t g = panels < cap ? panels : cap;
    return (int)(g < 1 ? 1 : g);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

BwdWork carve(void *ws, int64_t m, int np)
{
    BwdWork b;
    const int nt = np / 16;
    const int64_t E = (int64_t)nt * nt * 256;
    b.nwg = bwd_grid(m);
    b.nlvl2 = (b.nwg + 31) / 32;
    char *c = static_cast<char *>(ws);
    b.partials = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)(b.nwg * E));
    b.lvl2 = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)(b.nlvl2 * E));
    b.C = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)np * np);
    b.RT = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)np * np);
    b.dinv = reinterpret_cast<double *>(c);
    return b;
}

}  // namespace

size_t backward_ws_bytes(int64_t m, int n)
{
    const int np = padded_n(n);
    const int nt = np / 16;
    const int64_t E = (int64_t)nt * nt * 256;
    const int nwg = bwd_grid(m);
    const int nl = (nwg + 31) / 32;
    return align256(sizeof(double) * (size_t)(nwg * E)) + align256(sizeof(double) * (size_t)(nl * E)) +
           2 * align256(sizeof(double) * (size_t)np * np) + align256(sizeof(double) * (size_t)np) + 256;
}

// G = dQ^T Q over a contiguous share of 16-row panels; wave w owns tiles t = w + u * WAVES of
// the full NT x NT tile grid (t = I * NT + J).
template <int NP, int WAVES>
__global__ void __launch_bounds__(WAVES * 64)
k_bwd_gram(int64_t m, int n, const double *Q, int64_t ldq, const double *dQ, int64_t lddq,
           double *__restrict__ partials)
{
    constexpr int NT = NP / 16;
    constexpr int T = NT * NT;
    constexpr int TPW = (T + WAVES - 1) / WAVES;
    constexpr int PR = 16;
    constexpr int S = NP + 1;
    __shared__ double qs[PR * S], ds[PR * S];
    const int nthr = WAVES * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t npanels = (m + PR - 1) / PR;
    const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    d4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
    for (int64_t pn = p0; pn < p1; ++pn) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < PR * NP; idx += nthr) {
            const int rr = idx / NP, c = idx % NP;
            const int64_t row = pn * PR + rr;
            const bool ok = row < m && c < n;
            qs[rr * S + c] = ok ? Q[row * ldq + c] : 0.0;
            ds[rr * S + c] = ok ? dQ[row * lddq + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PR / 4; ++s) {
            const int off = (4 * s + (lane >> 4)) * S + (lane & 15);
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int t = wv + u * WAVES;
                if (t < T) {
                    const int I = t / NT, J = t % NT;
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ds[off + 16 * I], qs[off + 16 * J], acc[u], 0, 0, 0);
                }
            }
        }
    }
    double *out = partials + (int64_t)blockIdx.x * T * 256;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wv + u * WAVES;
        if (t < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[t * 256 + r * 64 + lane] = acc[u][r];
        }
    }
}

__global__ void __launch_bounds__(256)
k_bwd_reduce(const double *__restrict__ partials, double *__restrict__ lvl2, int nparts, int64_t elems)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= elems) return;
    const int g = blockIdx.y;
    const int p0 = 32 * g, p1 = (p0 + 32 < nparts) ? p0 + 32 : nparts;
    double s = 0.0;
    for (int q = p0; q < p1; ++q) s += partials[(int64_t)q * elems + e];
    lvl2[(int64_t)g * elems + e] = s;
}

// M = R dR^T - G and C = copyltu(M); padded transposed R and reciprocal diagonal.
template <int NP>
__global__ void __launch_bounds__(256)
k_bwd_small(BwdWork b, int n, const double *R, int64_t ldr, const double *dR, int64_t lddr,
            int have_dq)
{
    constexpr int NT = NP / 16;
    const int64_t E = (int64_t)NT * NT * 256;
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int i = idx / NP, k = idx % NP;
        // RT[k][i] = R[i][k]
        double v;
        if (i < n && k < n)
            v = (k >= i) ? R[(int64_t)i * ldr + k] : 0.0;
        else
            v = (i == k) ? 1.0 : 0.0;
        b.RT[k * NP + i] = v;
        b.C[idx] = 0.0;
    }
    for (int i = threadIdx.x; i < NP; i += blockDim.x) b.dinv[i] = (i < n) ? 1.0 / R[(int64_t)i * ldr + i] : 1.0;
    __syncthreads();
    // M_ij needed for i >= j only (copyltu keeps the lower triangle and mirrors it)
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        if (i < j) continue;
        double v = 0.0;
        if (dR) {
            // (R dR^T)_ij = sum_k R_ik dR_jk over k >= max(i, j) = i
            for (int k = i; k < n; ++k) v = __builtin_fma(R[(int64_t)i * ldr + k], dR[(int64_t)j * lddr + k], v);
        }
        double g = 0.0;
        if (have_dq) {
            const int I = i / 16, J = j / 16, ii = i % 16, jj = j % 16;
            // element (ii, jj) of tile (I, J) in the FP64 accumulator layout
            const int lane = jj + 16 * (ii % 4), r = ii / 4;
            const int64_t e = (int64_t)(I * NT + J) * 256 + r * 64 + lane;
            for (int gq = 0; gq < b.nlvl2; ++gq) g += b.lvl2[(int64_t)gq * E + e];
        }
        const double mij = v - g;
        b.C[i * NP + j] = mij;
        b.C[j * NP + i] = mij;
    }
}

// Per row: y = dq + q C (block J of 64 columns at a time, written into dX), then the back
// substitution dx R^T = y from the last column block to the first.
template <int NP>
__global__ void __launch_bounds__(256)
k_bwd_rows(BwdWork b, int64_t m, int n, const double *Q, int64_t ldq, const double *dQ,
           int64_t lddq, double *dX, int64_t lddx)
{
    constexpr int NB = (NP + 63) / 64;
    constexpr int BW = NP < 64 ? NP : 64;
    for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < m; row += (int64_t)gridDim.x * 256) {
        const double *q = Q + row * ldq;
        const double *dq = dQ ? dQ + row * lddq : nullptr;
        double *dx = dX + row * lddx;
        for (int J = 0; J < NB; ++J) {
            double t[BW];
#pragma unroll
            for (int c = 0; c < BW; ++c) t[c] = 0.0;
            for (int k = 0; k < n; ++k) {
                const double qk = q[k];
                const double *ck = b.C + (int64_t)k * NP + BW * J;
#pragma unroll
                for (int c = 0; c < BW; ++c) t[c] = __builtin_fma(qk, ck[c], t[c]);
            }
#pragma unroll
            for (int c = 0; c < BW; ++c) {
                const int col = BW * J + c;
                if (col < n) dx[col] = (dq ? dq[col] : 0.0) + t[c];
            }
        }
        for (int J = NB - 1; J >= 0; --J) {
            double t[BW];
#pragma unroll
            for (int c = 0; c < BW; ++c) t[c] = (BW * J + c < n) ? dx[BW * J + c] : 0.0;
            for (int K = NB - 1; K > J; --K) {
                for (int kk = BW - 1; kk >= 0; --kk) {
                    const int k = BW * K + kk;
                    const double xk = (k < n) ? dx[k] : 0.0;
                    const double *rk = b.RT + (int64_t)k * NP + BW * J;  // R[BW J + c][k]
#pragma unroll
                    for (int c = 0; c < BW; ++c) t[c] = __builtin_fma(-xk, rk[c], t[c]);
                }
            }
#pragma unroll
            for (int jj = BW - 1; jj >= 0; --jj) {
                const int j = BW * J + jj;
                const double xj = t[jj] * b.dinv[j];
                t[jj] = xj;
                const double *rj = b.RT + (int64_t)j * NP + BW * J;
#pragma unroll
                for (int c = 0; c < jj; ++c) t[c] = __builtin_fma(-xj, rj[c], t[c]);
            }
#pragma unroll
            for (int c = 0; c < BW; ++c)
                if (BW * J + c < n) dx[BW * J + c] = t[c];
        }
    }
}

template <int NP, int WAVES>
static hipError_t bwd_impl(hipStream_t s, int64_t m, int n, const double *Q, int64_t ldq,
                           const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                           const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws)
{
    BwdWork b = carve(ws, m, NP);
    constexpr int NT = NP / 16;
    const int64_t E = (int64_t)NT * NT * 256;
    if (dQ) {
        prof_before(s, "bwd_gram");
        hipLaunchKernelGGL((k_bwd_gram<NP, WAVES>), dim3(b.nwg), dim3(WAVES * 64), 0, s, m, n, Q, ldq, dQ,
                           lddq, b.partials);
        prof_after(s);
        prof_before(s, "bwd_reduce");
        hipLaunchKernelGGL(k_bwd_reduce, dim3((unsigned)((E + 255) / 256), (unsigned)b.nlvl2), dim3(256), 0,
                           s, b.partials, b.lvl2, b.nwg, E);
        prof_after(s);
    }
    prof_before(s, "bwd_small");
    hipLaunchKernelGGL((k_bwd_small<NP>), dim3(1), dim3(256), 0, s, b, n, R, ldr, dR, lddr, dQ ? 1 : 0);
    prof_after(s);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t blocks = (m + 255) / 256;
    if (blocks > 4 * (int64_t)cus) blocks = 4 * (int64_t)cus;
    if (blocks < 1) blocks = 1;
    prof_before(s, "bwd_rows");
    hipLaunchKernelGGL((k_bwd_rows<NP>), dim3((unsigned)blocks), dim3(256), 0, s, b, m, n, Q, ldq, dQ, lddq,
                       dX, lddx);
    prof_after(s);
    return hipGetLastError();
}

hipError_t launch_backward(hipStream_t s, int64_t m, int n, const double *Q, int64_t ldq,
                           const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                           const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws)
{
    switch (padded_n(n)) {
    case 16: return bwd_impl<16, 1>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 32: return bwd_impl<32, 4>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 64: return bwd_impl<64, 4>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 128: return bwd_impl<128, 8>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 256: return bwd_impl<256, 16>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    }
    return hipErrorInvalidValue;
}

}  // namespace scqr
