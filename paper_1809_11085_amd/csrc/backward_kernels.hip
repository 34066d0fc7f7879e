// QR adjoint on gfx950 (reverse-mode derivative of X -> (Q, R), thin QR with positive diag):
//   G = dQ^T Q (split-m, FP64 MFMA, fixed-order reduction),
//   M = R dR^T - G,  C = copyltu(M)  (C_ij = M_{max(i,j), min(i,j)}),
//   Y = dQ + Q C (FP64 MFMA product with C staged in LDS),
//   dX R^T = Y solved row by row (back substitution in blocked order: off-diagonal 16x16 blocks
//   on FP64 MFMA, diagonal blocks per lane), in place in dX.
#include "scqr_internal.h"

namespace scqr {

namespace {

struct BwdWork {
    double *partials;  // nwg x NT(NT+1)/2 * 256 (tiles I >= J of G)
    double *lvl2;      // nlvl2 x NT(NT+1)/2 * 256
    double *C;         // np x np
    double *Rp;        // np x np: R with identity padding (upper triangle)
    double *dinv;      // np
    double *Rsplit;    // np = 256: diagonal 128 x 128 blocks of R and their reciprocal diagonals
    int nwg, nlvl2;
};

int bwd_grid(int64_t m)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t panels = (m + 31) / 32;
    const int64_t cap = 2 * (int64_t)(cus > 0 ? cus : 256);
    const int64_t g = panels < cap ? panels : cap;
    return (int)(g < 1 ? 1 : g);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t split_doubles(int np) { return np == 256 ? 2 * 128 * 128 + 256 : 0; }

BwdWork carve(void *ws, int64_t m, int np)
{
    BwdWork b;
    const int nt = np / 16;
    const int64_t E = (int64_t)nt * (nt + 1) / 2 * 256;
    b.nwg = bwd_grid(m);
    b.nlvl2 = (b.nwg + 31) / 32;
    char *c = static_cast<char *>(ws);
    b.partials = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)(b.nwg * E));
    b.lvl2 = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)(b.nlvl2 * E));
    b.C = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)np * np);
    b.Rp = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)np * np);
    b.dinv = reinterpret_cast<double *>(c);
    c += align256(sizeof(double) * (size_t)np);
    b.Rsplit = split_doubles(np) ? reinterpret_cast<double *>(c) : nullptr;
    return b;
}

}  // namespace

size_t backward_ws_bytes(int64_t m, int n)
{
    const int np = padded_n(n);
    const int nt = np / 16;
    const int64_t E = (int64_t)nt * (nt + 1) / 2 * 256;
    const int nwg = bwd_grid(m);
    const int nl = (nwg + 31) / 32;
    return align256(sizeof(double) * (size_t)(nwg * E)) + align256(sizeof(double) * (size_t)(nl * E)) +
           2 * align256(sizeof(double) * (size_t)np * np) + align256(sizeof(double) * (size_t)np) +
           align256(sizeof(double) * split_doubles(np)) + 256;
}

// G = dQ^T Q over a contiguous share of panels (64 rows, 16 for n = 256) staged in LDS with the
// next panel's loads issued before the current panel's MFMAs.  Only the tiles I >= J are formed
// (C reads G at (max(i, j), min(i, j))); tile t = I (I + 1) / 2 + J, and wave w owns the tiles
// t = w, w + WAVES, ...
template <int NP>
__global__ void __launch_bounds__(NP == 256 ? 1024 : (NP >= 128 ? 512 : 256))
k_bwd_gram(int64_t m, int n, const double *__restrict__ Q, int64_t ldq, const double *__restrict__ dQ,
           int64_t lddq, double *__restrict__ partials)
{
    constexpr int WV = NP == 256 ? 16 : (NP >= 128 ? 8 : 4);
    constexpr int NTH = 64 * WV;
    // 16 rows and 16 waves at n = 256: 9 tile accumulators and both prefetched panels fit 128
    // registers, four waves per SIMD
    constexpr int PR = NP == 256 ? 16 : 64;
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int TPW = (T + WV - 1) / WV;
    constexpr int S = lds_stride_gram(NP);
    constexpr int PP = PR * NP / 2 / NTH;
    static_assert(PP >= 1 && (PR * NP / 2) % NTH == 0, "panel must split over the workgroup");
    __shared__ __attribute__((aligned(16))) double qs[PR * S];
    __shared__ __attribute__((aligned(16))) double ds[PR * S];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t npanels = (m + PR - 1) / PR;
    const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
    int64_t p0 = (int64_t)blockIdx.x * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    if (p0 > p1) p0 = p1;

    d4 acc[TPW];
    int ti[TPW], tj[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
        const int tt = wv + WV * u < T ? wv + WV * u : 0;
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= tt) ++I;
        ti[u] = 16 * I;
        tj[u] = 16 * (tt - I * (I + 1) / 2);
    }
    double2 pq[PP], pd[PP];
    auto pair_at = [&](const double *M, int64_t ld, int64_t row, int c) -> double2 {
        double a = 0.0, b = 0.0;
        if (row < m) {
            const gview<const double> src = as_global(M) + row * ld + c;
            if (c < n) a = src[0];
            if (c + 1 < n) b = src[1];
        }
        return make_double2(a, b);
    };
    auto load_panel = [&](int64_t pnl) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + NTH * i;
            const int64_t row = pnl * PR + e2 / (NP / 2);
            const int c = 2 * (e2 % (NP / 2));
            pq[i] = pair_at(Q, ldq, row, c);
            pd[i] = pair_at(dQ, lddq, row, c);
        }
    };
    if (p0 < p1) load_panel(p0);
    for (int64_t pn = p0; pn < p1; ++pn) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + NTH * i;
            const int o = (e2 / (NP / 2)) * S + 2 * (e2 % (NP / 2));
            *reinterpret_cast<double2 *>(qs + o) = pq[i];
            *reinterpret_cast<double2 *>(ds + o) = pd[i];
        }
        __syncthreads();
        if (pn + 1 < p1) load_panel(pn + 1);
        const int off = (lane >> 4) * S + (lane & 15);
#pragma unroll 2
        for (int s4 = 0; s4 < PR / 4; ++s4) {
            const double *dr = ds + off + 4 * s4 * S;
            const double *qr = qs + off + 4 * s4 * S;
#pragma unroll
            for (int u = 0; u < TPW; ++u)
                if (wv + WV * u < T) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(dr[ti[u]], qr[tj[u]], acc[u], 0, 0, 0);
        }
    }
    double *out = partials + (int64_t)blockIdx.x * T * 256;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int tt = wv + WV * u;
        if (tt < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[tt * 256 + r * 64 + lane] = acc[u][r];
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

// One thread per entry (i, j) of the padded n x n matrices:
//   C_ij = M_ab with (a, b) = (max(i, j), min(i, j)),  M_ab = sum_{k >= a} R_ak dR_bk - G_ab,
// the padded R (identity padding) and the reciprocal diagonal of R.
template <int NP>
__global__ void __launch_bounds__(256)
k_bwd_c(BwdWork b, int n, const double *R, int64_t ldr, const double *dR, int64_t lddr, int have_dq)
{
    constexpr int NT = NP / 16;
    const int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= NP * NP) return;
    const int i = idx / NP, j = idx % NP;
    double rv;
    if (i < n && j < n)
        rv = (j >= i) ? R[(int64_t)i * ldr + j] : 0.0;
    else
        rv = (i == j) ? 1.0 : 0.0;
    b.Rp[idx] = rv;
    if (idx < NP) b.dinv[idx] = (idx < n) ? 1.0 / R[(int64_t)idx * ldr + idx] : 1.0;
    double c = 0.0;
    if (i < n && j < n) {
        const int a = i > j ? i : j, bb = i > j ? j : i;
        double v = 0.0;
        if (dR) {
            // (R dR^T)_ab = sum_k R_ak dR_bk over k >= max(a, b) = a, in increasing k
            const double *ra = R + (int64_t)a * ldr, *db = dR + (int64_t)bb * lddr;
            int k = a;
            for (; k + 8 <= n; k += 8) {
                double x[8], y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    x[u] = ra[k + u];
                    y[u] = db[k + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) v = __builtin_fma(x[u], y[u], v);
            }
            for (; k < n; ++k) v = __builtin_fma(ra[k], db[k], v);
        }
        double g = 0.0;
        if (have_dq) {
            // element (a % 16, bb % 16) of tile (a / 16, bb / 16) in the FP64 accumulator layout
            const int ii = a % 16, jj = bb % 16;
            const int I = a / 16, J = bb / 16;
            const int64_t e = (int64_t)(I * (I + 1) / 2 + J) * 256 + (ii / 4) * 64 + jj + 16 * (ii % 4);
            for (int gq = 0; gq < b.nlvl2; ++gq) g += b.lvl2[(int64_t)gq * E + e];
        }
        c = v - g;
    }
    b.C[idx] = c;
}

template <int NP>
static hipError_t bwd_impl(hipStream_t s, int64_t m, int n, const double *Q, int64_t ldq,
                           const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                           const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws)
{
    BwdWork b = carve(ws, m, NP);
    constexpr int NT = NP / 16;
    constexpr int NTH = NP == 256 ? 1024 : (NP >= 128 ? 512 : 256);
    const int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    if (dQ) {
        prof_before(s, "bwd_gram");
        hipLaunchKernelGGL((k_bwd_gram<NP>), dim3(b.nwg), dim3(NTH), 0, s, m, n, Q, ldq, dQ, lddq, b.partials);
        prof_after(s);
        prof_before(s, "bwd_reduce");
        hipLaunchKernelGGL(k_bwd_reduce, dim3((unsigned)((E + 255) / 256), (unsigned)b.nlvl2), dim3(256), 0,
                           s, b.partials, b.lvl2, b.nwg, E);
        prof_after(s);
    }
    prof_before(s, "bwd_c");
    hipLaunchKernelGGL((k_bwd_c<NP>), dim3((NP * NP + 255) / 256), dim3(256), 0, s, b, n, R, ldr, dR, lddr,
                       dQ ? 1 : 0);
    prof_after(s);
    prof_before(s, "bwd_y");
    hipError_t e = launch_mm(s, NP, m, n, n, Q, ldq, b.C, NP, dQ, lddq, dX, lddx);
    prof_after(s);
    if (e != hipSuccess) return e;
    prof_before(s, "bwd_solve");
    e = launch_solve_t(s, NP, m, n, dX, lddx, b.Rp, b.dinv, b.Rsplit);
    prof_after(s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_backward(hipStream_t s, int64_t m, int n, const double *Q, int64_t ldq,
                           const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                           const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws)
{
    switch (padded_n(n)) {
    case 16: return bwd_impl<16>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 32: return bwd_impl<32>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 64: return bwd_impl<64>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 128: return bwd_impl<128>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    case 256: return bwd_impl<256>(s, m, n, Q, ldq, R, ldr, dQ, lddq, dR, lddr, dX, lddx, ws);
    }
    return hipErrorInvalidValue;
}

}  // namespace scqr
