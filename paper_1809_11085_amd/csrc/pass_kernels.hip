// Row-panel kernels of one Cholesky QR pass on gfx950:
//   * Gram A = X^T X (eq:gram) as a split-m SYRK on FP64 MFMA (16x16x4), upper 16x16 tiles;
//   * Q = X R~^{-1} by row-wise forward substitution (Algorithm 1 line 4, the row-wise solve
//     whose backward error equation (eq:backward2) models), fused with the Gram of the new Q
//     so that a pass reads its input from HBM once and writes Q once;
//   * the oblique Gram X^T B X for tridiagonal B (Algorithm 4) with one halo row per panel;
//   * a binary32 MFMA Gram for the FP32-first option;
//   * a fixed-order reduction of the per-workgroup partial Grams.
// Every reduction order is fixed, so results are bitwise reproducible run to run.
#include "scqr_internal.h"

namespace scqr {

// ------------------------------------------------------------------------------------------
// Control-block predicates.  pass == 0: unconditional; pass < 0: only when the FP32-first
// pass must be redone in binary64; pass > 0: only when R~ of that pass is ready and the
// schedule is still active.
__device__ __forceinline__ bool gate(const Ctl *c, int pass)
{
    if (pass == 0) return true;
    if (pass < 0) return c->active && c->redo_fp64;
    return c->active && c->pass == pass;
}
// The Gram of the Q produced by pass `pass` is needed unless that pass is the last one.
__device__ __forceinline__ bool gram_needed(const Ctl *c, int pass, int final_gram)
{
    if (pass <= 0) return true;
    return final_gram || c->last != pass;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------------------------------
// Fused pass for n <= 64.  Each wave owns panels of PR rows staged in a per-wave LDS buffer
// (coalesced 16-byte global loads and stores).  Q = X R~^{-1} is a blocked row-wise
// substitution over 16-column blocks J:
//   T_J = X_J - sum_{K<J} Q_K R~_KJ   on FP64 MFMA, with -R~_KJ staged once per workgroup in
//                                     LDS in the 4x16 B-operand layout;
//   Q_J = T_J R~_JJ^{-1}              one row per lane, forward substitution against the 16x16
//                                     diagonal block (wave-uniform scalar loads), multiplying by
//                                     the reciprocal diagonal.
// Each q_ij is thus x_ij minus the products q_ik r_kj, k < j, divided by r_jj: a row-wise
// substitution in blocked order, whose backward error is bounded row by row as in (eq:backward2).
// The solved panel then feeds the FP64 MFMA Gram (all upper 16x16 tiles in registers).
//   MODE 0: Gram of X only.  MODE 1: TRSM + Gram.  MODE 2: TRSM only.  MODE 3: the transposed
//   solve x R~^T = y row by row (back substitution in blocked order, for the QR adjoint).
//   MODE 5 (minimum traffic, NP <= 32): Rt and dinv are the factor history; the panel of X is
//   solved against the factors of passes 1 .. pass in turn, exactly as the stored-Q passes
//   solve it one pass at a time, so the panel equals that pass's Q bit for bit.  Q is written
//   only when this pass is the last one; the Gram follows as in MODE 1.
//   F32: Gram in binary32 MFMA, each panel (one chain of f32_chain_rows(NP) = PR rows) added to the
//        binary64 tiles after the panel (MODE 0 only).
//   VEC: n even, even leading dimensions and 16-byte aligned X, Q (pairs of doubles per access).
//   PR: rows per panel (32: 8 waves per workgroup, 64: 4 waves).
//   BATCH false: one problem; the waves of all workgroups interleave over its panels.
//   BATCH true: workgroup b takes task b of the device task table (a row range of one
//   instance); the problem, factor and control block come from the instance's descriptor.
//   Workgroup b's partial Gram goes to partials + b * T * 256.
template <int NP, int MODE, bool F32, bool VEC, int PR, bool BATCH>
__global__ void __launch_bounds__(PR == 64 ? 256 : 512)
k_pass_tile(Problem p, double *__restrict__ Qout, const double *__restrict__ Rt,
            const double *__restrict__ dinv, double *__restrict__ partials,
            const Ctl *__restrict__ ctl, int pass, int final_gram,
            const BatchInst *__restrict__ insts, const BatchTask *__restrict__ tasks)
{
    int64_t pfirst = 0, pend = 0;
    if constexpr (BATCH) {
        // batched: workgroup b processes task b (rows [r0, r1) of one instance); pass > 1
        // reads the instance's Q
        const BatchTask tk = load_cview(tasks + blockIdx.x);
        const BatchInst I = load_cview(insts + tk.inst);
        p = I.p;
        if (pass > 1) {
            p.X = p.Q;
            p.ldx = p.ldq;
        }
        Qout = p.Q;
        Rt = factor_of(I.w, NP, pass);
        dinv = dinv_of(I.w, NP, pass);
        ctl = I.w.ctl;
        pfirst = tk.r0 / PR;
        pend = (tk.r1 + PR - 1) / PR;
    }
    // Qout == p.Q, a restrict parameter so that the factor loads stay scalar.  When Q aliases
    // X every row is read before it is written by the same wave.
    constexpr int WAVES = PR == 64 ? 4 : 8;
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int NOFF = NT * (NT - 1) / 2;
    // LDS row stride (doubles): 2 S = 4 (mod 64) dwords, so that one row per lane (per-lane
    // substitution, 16-byte reads) and 16 rows by 4 consecutive columns (MFMA A operands) are
    // free of bank conflicts on the 64 banks.  Where a half-wave reads two rows across 16
    // consecutive columns (MFMA result tiles and Gram operands), the rows are chosen 8 apart
    // (2 S * 8 = 32 mod 64), which puts them on opposite halves of the banks:
    //   MFMA row index i = lk + 4 r of a 16-row group <-> panel row rowperm(i) = 8 (i & 1) +
    //   4 ((i >> 1) & 1) + (i >> 2);   Gram k-step s, lane row lk <-> panel row (s & 7) + 8 lk +
    //   32 (s >> 3).  Every row is still solved and summed exactly once.
    constexpr int S = NP + 2;
    constexpr int PANEL = PR * S;
    constexpr int LDSZ = (WAVES * PANEL > T * 256) ? WAVES * PANEL : T * 256;
    constexpr int PP = PR * NP / 2 / 64;  // double pairs per lane per panel
    static_assert((PR * NP / 2) % 64 == 0, "panel must split evenly over a wave");
    static_assert(PR % 32 == 0, "Gram row mapping covers 32-row blocks");
    static_assert(!F32 || PR == f32_chain_rows(NP), "a binary32 chain is one panel");
    // MODE 5 holds -R~_KJ of every factor it applies (one per pass up to this one) in dynamic
    // LDS of pass * BLF doubles
    static_assert(MODE != 5 || (NP <= 32 && !BATCH && !F32), "minimum-traffic passes: n <= 32, one problem");
    constexpr int BLF = NOFF * 4 * 64;
    constexpr int BL = (MODE >= 1 && MODE != 5 && NOFF > 0) ? BLF : 1;
    __shared__ __attribute__((aligned(16))) double lds[LDSZ];
    __shared__ double bl_s[BL];
    extern __shared__ double bl_dyn[];
    double *const bl = MODE == 5 ? bl_dyn : bl_s;

    if (!gate(ctl, pass)) return;
    const bool want_gram = (MODE == 0) || ((MODE == 1 || MODE == 5) && gram_needed(ctl, pass, final_gram));
    // factors applied to each panel, and whether the panel is stored
    const int nfac = MODE == 5 ? pass : 1;
    const bool store_q = MODE != 5 || ctl->last == pass;

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // single problem: waves interleaved over all panels; batched: the task's panel range
    const int64_t W = BATCH ? (int64_t)WAVES : (int64_t)gridDim.x * WAVES;
    const int64_t npanels = BATCH ? pend : (p.m + PR - 1) / PR;
    const int n = p.n;
    double *P = lds + wv * PANEL;
    const int li = lane & 15, lk = lane >> 4;
    const int pli = 8 * (li & 1) + 4 * ((li >> 1) & 1) + (li >> 2);  // rowperm(li)
    const int plk = 8 * (lk & 1) + 4 * (lk >> 1);                    // rowperm(lk + 4 r) - r

    // -R~_KJ (K < J) in the B-operand layout, one 64-entry vector per (block pair, k-step):
    // entry l holds -r[16K + 4s + l/16][16J + l%16].
    if constexpr (MODE >= 1 && NOFF > 0) {
        for (int idx = threadIdx.x; idx < BLF * nfac; idx += WAVES * 64) {
            const int f = idx / BLF;  // factor (MODE 5); 0 otherwise
            const int l = idx & 63, s4 = (idx >> 6) & 3, pi = (idx - f * BLF) >> 8;
            int J = 1, K = pi;
            while (K >= J) {
                K -= J;
                ++J;
            }
            // MODE 3 uses the transposed blocks: entry l holds -r[16K + l%16][16J + 4s + l/16]
            const int e = f * NP * NP +
                          (MODE == 3 ? (16 * K + (l & 15)) * NP + 16 * J + 4 * s4 + (l >> 4)
                                     : (16 * K + 4 * s4 + (l >> 4)) * NP + 16 * J + (l & 15));
            bl[idx] = -(BATCH ? as_cview(Rt)[e] : Rt[e]);
        }
        __syncthreads();
    }

    d4 acc[T];
#pragma unroll
    for (int u = 0; u < T; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};

    // X panel pn -> registers (pairs of doubles, coalesced); issued one panel ahead, right after
    // the current panel is staged in LDS, so that the loads of the next panel overlap the whole
    // substitution, Q store and Gram of the current one.
    // VEC: every pair a lane moves lies in column cl, rows rl + i * (128 / NP) of the panel;
    // buffer accesses return zeros (loads) or are dropped (stores) past the end of the matrix,
    // and padding columns (cl >= n) use an offset outside the resource.
    double2 pre[PP];
    // a pass streams X and Q once (non-temporal: measured 0.90 -> 0.86 ms for the fused pass and
    // 0.42 -> 0.34 ms for the first Gram at 2^22 x 64; the c4 batch 66-67 -> 63.5 ms)
    constexpr int CPOL = kBufStream;
    const int cl = 2 * (lane % (NP / 2)), rl = lane / (NP / 2);
    constexpr int RSTEP = 128 / NP;
    const uint32_t offx = cl < n ? (uint32_t)((rl * p.ldx + cl) * 8) : kBufOut;
    const uint32_t dxs = (uint32_t)(RSTEP * p.ldx * 8);
    auto load_panel = [&](int64_t pnl) {
        const int64_t rb = pnl * PR;
        if constexpr (VEC) {
            const __amdgpu_buffer_rsrc_t rs = rows_rsrc(p.X, p.ldx, rb, p.m, n);
#pragma unroll
            for (int i = 0; i < PP; ++i) pre[i] = buf_load2<CPOL>(rs, offx + (uint32_t)i * dxs);
            return;
        }
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = lane + 64 * i;
            const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
            const int64_t row = rb + r;
            {
                double a = 0.0, b = 0.0;
                if (row < p.m) {
                    const double *src = p.X + row * p.ldx + c;
                    if (c < n) a = src[0];
                    if (c + 1 < n) b = src[1];
                }
                pre[i] = make_double2(a, b);
            }
        }
    };
    int64_t pn = (BATCH ? pfirst : (int64_t)blockIdx.x * WAVES) + wv;
    if (pn < npanels) load_panel(pn);
    for (; pn < npanels; pn += W) {
        const int64_t r0 = pn * PR;
        const int64_t nxt = pn + W;
        // ---- staged X panel -> LDS
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = lane + 64 * i;
            const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
            *reinterpret_cast<double2 *>(P + r * S + c) = pre[i];
        }
        wave_sync();
        if (nxt < npanels) load_panel(nxt);
        if (MODE >= 1) {
            // The opaque zero keeps the diagonal-block loads inside the panel loop (as scalar
            // loads of a 4 KB working set) instead of hoisting them into spilled registers.
            const int64_t off = pn & (int64_t)p.zero;
            if constexpr (MODE == 3) {
                // y = x R~^T solved for x, blocks from the last to the first:
                //   T_J = Y_J - sum_{K>J} X_K R~_JK^T  (FP64 MFMA),
                //   x_k = t_k / r_kk, then t_j -= r_jk x_k for j < k (per lane, back substitution)
#pragma unroll
                for (int JB = NT - 1; JB >= 0; --JB) {
                    if (JB < NT - 1) {
#pragma unroll
                        for (int g = 0; g < PR / 16; ++g) {
                            double *blk = P + (16 * g + plk) * S + 16 * JB + li;
                            d4 d;
#pragma unroll
                            for (int r = 0; r < 4; ++r) d[r] = blk[r * S];
                            const double *arow = P + (16 * g + pli) * S + lk;
#pragma unroll
                            for (int J2 = JB + 1; J2 < NT; ++J2) {
                                const int pi = J2 * (J2 - 1) / 2 + JB;
#pragma unroll
                                for (int s4 = 0; s4 < 4; ++s4)
                                    d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * J2 + 4 * s4],
                                                                             bl[(pi * 4 + s4) * 64 + lane], d, 0, 0, 0);
                            }
#pragma unroll
                            for (int r = 0; r < 4; ++r) blk[r * S] = d[r];
                        }
                        wave_sync();
                    }
                    if (lane < PR) {
                        double *mr = P + lane * S + 16 * JB;
                        double t[16];
#pragma unroll
                        for (int c = 0; c < 16; c += 2) {
                            const double2 v = *reinterpret_cast<const double2 *>(mr + c);
                            t[c] = v.x;
                            t[c + 1] = v.y;
                        }
                        int64_t offk = off;
#pragma unroll
                        for (int k = 15; k >= 0; --k) {
                            if (((15 - k) & 1) == 0) asm volatile("" : "+s"(offk));
                            const double *Rd = Rt + offk + (16 * JB) * NP + 16 * JB;
                            const double qk = t[k] * dinv[offk + 16 * JB + k];
                            t[k] = qk;
#pragma unroll
                            for (int j = 0; j < k; ++j) t[j] = __builtin_fma(-qk, Rd[j * NP + k], t[j]);
                        }
#pragma unroll
                        for (int c = 0; c < 16; c += 2) *reinterpret_cast<double2 *>(mr + c) = make_double2(t[c], t[c + 1]);
                    }
                    wave_sync();
                }
            } else {
            // MODE 5: factors 1 .. pass in turn (a runtime loop around the same blocked solve)
            for (int f = 0; f < nfac; ++f) {
                const double *Rtf = Rt + f * (NP * NP);
                const double *dvf = dinv + f * NP;
                const double *blf = bl + f * BLF;
                int pi0 = 0;
#pragma unroll
                for (int J = 0; J < NT; ++J) {
                    if (J > 0) {
#pragma unroll
                        for (int g = 0; g < PR / 16; ++g) {
                            double *blk = P + (16 * g + plk) * S + 16 * J + li;
                            d4 d;
#pragma unroll
                            for (int r = 0; r < 4; ++r) d[r] = blk[r * S];
                            const double *arow = P + (16 * g + pli) * S + lk;
                            int pi = pi0;
#pragma unroll
                            for (int K = 0; K < J; ++K, ++pi)
#pragma unroll
                                for (int s4 = 0; s4 < 4; ++s4)
                                    d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * K + 4 * s4],
                                                                             blf[(pi * 4 + s4) * 64 + lane], d, 0, 0, 0);
#pragma unroll
                            for (int r = 0; r < 4; ++r) blk[r * S] = d[r];
                        }
                        pi0 += J;
                        wave_sync();
                    }
                    if (lane < PR) {
                        double *mr = P + lane * S + 16 * J;
                        double t[16];
#pragma unroll
                        for (int c = 0; c < 16; c += 2) {
                            const double2 v = *reinterpret_cast<const double2 *>(mr + c);
                            t[c] = v.x;
                            t[c + 1] = v.y;
                        }
                        int64_t offk = off;
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            // re-laundered every two rows: later rows' scalar loads may not be
                            // hoisted above earlier rows' work (they would exhaust the SGPRs)
                            if ((k & 1) == 0) asm volatile("" : "+s"(offk));
                            if constexpr (BATCH) {
                                const cview<double> Rd = as_cview(Rtf) + offk + (16 * J) * NP + 16 * J;
                                const double qk = t[k] * as_cview(dvf)[offk + 16 * J + k];
                                t[k] = qk;
#pragma unroll
                                for (int j = k + 1; j < 16; ++j) t[j] = __builtin_fma(-qk, Rd[k * NP + j], t[j]);
                            } else {
                                const double *Rd = Rtf + offk + (16 * J) * NP + 16 * J;
                                const double qk = t[k] * dvf[offk + 16 * J + k];
                                t[k] = qk;
#pragma unroll
                                for (int j = k + 1; j < 16; ++j) t[j] = __builtin_fma(-qk, Rd[k * NP + j], t[j]);
                            }
                        }
#pragma unroll
                        for (int c = 0; c < 16; c += 2) *reinterpret_cast<double2 *>(mr + c) = make_double2(t[c], t[c + 1]);
                    }
                    wave_sync();
                }
            }
            }
            // ---- Q panel -> HBM
            if (store_q) {
                if constexpr (VEC) {
                    const __amdgpu_buffer_rsrc_t rq = rows_rsrc(Qout, p.ldq, r0, p.m, n);
                    const uint32_t offq = cl < n ? (uint32_t)((rl * p.ldq + cl) * 8) : kBufOut;
                    const uint32_t dqs = (uint32_t)(RSTEP * p.ldq * 8);
#pragma unroll
                    for (int i = 0; i < PP; ++i)
                        buf_store2<CPOL>(rq, offq + (uint32_t)i * dqs,
                                   *reinterpret_cast<const double2 *>(P + (rl + RSTEP * i) * S + cl));
                } else {
#pragma unroll
                    for (int i = 0; i < PP; ++i) {
                        const int e2 = lane + 64 * i;
                        const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
                        const int64_t row = r0 + r;
                        if (row < p.m && c < n) {
                            const double2 v = *reinterpret_cast<const double2 *>(P + r * S + c);
                            double *dst = Qout + row * p.ldq + c;
                            dst[0] = v.x;
                            if (c + 1 < n) dst[1] = v.y;
                        }
                    }
                }
            }
        }
        if (want_gram) {
            f4 acc32[F32 ? T : 1];
            if (F32) {
#pragma unroll
                for (int u = 0; u < (F32 ? T : 1); ++u) acc32[u] = (f4){0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int s = 0; s < PR / 4; ++s) {
                const double *src = P + ((s & 7) + 8 * lk + 32 * (s >> 3)) * S + li;
                if (F32) {
                    float op[NT];
#pragma unroll
                    for (int b = 0; b < NT; ++b) op[b] = (float)src[16 * b];
                    int tt = 0;
#pragma unroll
                    for (int I = 0; I < NT; ++I)
#pragma unroll
                        for (int J = I; J < NT; ++J, ++tt)
                            acc32[F32 ? tt : 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(op[I], op[J], acc32[F32 ? tt : 0], 0, 0, 0);
                } else {
                    double op[NT];
#pragma unroll
                    for (int b = 0; b < NT; ++b) op[b] = src[16 * b];
                    int tt = 0;
#pragma unroll
                    for (int I = 0; I < NT; ++I)
#pragma unroll
                        for (int J = I; J < NT; ++J, ++tt)
                            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], acc[tt], 0, 0, 0);
                }
            }
            if (F32) {
#pragma unroll
                for (int u = 0; u < T; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u][r] += (double)acc32[F32 ? u : 0][r];
            }
        }
        wave_sync();
    }
    if (!want_gram) return;

    // Fixed-order sum of the waves' tiles: (((w0 + w1) + w2) + ...).
    __syncthreads();
    double *red = lds;
    for (int w = 0; w < WAVES; ++w) {
        if (wv == w) {
#pragma unroll
            for (int u = 0; u < T; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = u * 256 + r * 64 + lane;
                    red[e] = (w == 0) ? acc[u][r] : red[e] + acc[u][r];
                }
        }
        __syncthreads();
    }
    double *out = partials + (int64_t)blockIdx.x * (T * 256);
    for (int e = threadIdx.x; e < T * 256; e += WAVES * 64) out[e] = red[e];
}

// ------------------------------------------------------------------------------------------
// Fused pass for 64 < n <= 128 (NP = 128).  A workgroup of 4 waves shares one 64-row panel in
// LDS.  Each wave solves its own 16 rows block by block: the off-diagonal 16x16 blocks on FP64
// MFMA against -R~_KJ held in LDS in the B-operand layout, then the diagonal block in the MFMA
// result layout with all 64 lanes (row broadcasts by DPP, per-lane coefficients r_kj / r_kk from
// an LDS table; diag_solve_steps).  The solved panel is written to Q, and wave w accumulates
// the upper Gram tiles t = w, w+4, ... over all 64 rows.  The next panel's loads are issued before the current one is solved.
//   MODE 1: substitution + Gram.  MODE 2: substitution only.  MODE 3: the transposed solve
//   x R~^T = y (back substitution in blocked order, for the QR adjoint).  MODE 4: substitution,
//   then X'_2 = X_2 - Q_1 R~_12 for the panel's rows (WideProd): wave w forms output columns
//   32 w .. 32 w + 31 from the solved panel in LDS and its slice of -R~_12 held in registers, with
//   the panel's X_2 loaded before the substitution.
//   The workgroup takes the 64-row panels [p0, p1).
// Lane K of every 16-lane row of the wave, broadcast to the whole row (DPP row_newbcast; every
// lane is written, so the old value is never used).
template <int K>
__device__ __forceinline__ double row_bcast(double v)
{
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xF, 0xF, true);
}

// Substitution inside a 16 x 16 diagonal block held in the MFMA result layout (lane l holds
// column l % 16 of rows l / 16 + 4 r): column K's value is final when step K runs; it is
// broadcast along the lane's row and column j takes -t_K c[K] (c = r_Kj / r_KK for the columns
// K still updates, 0 elsewhere).  FWD runs K = 0, 1, ..., 15, otherwise K = 15, ..., 0.  The
// reciprocal diagonal is applied by the caller after the last step.
// The first step is left to the compiler: its inputs come from MFMAs, whose read-after-write
// waits the compiler inserts.  Every later step reads values the previous step wrote on the VALU
// and takes the broadcast as a DPP operand of v_fmac_f64 (d -= bcast(d) c in one instruction with
// one rounding, the same value as the separate broadcast and FMA), after the two wait states a
// DPP read of a VALU result needs.
template <int K>
__device__ __forceinline__ void diag_step_dpp(d4 &d, double c)
{
    double a0 = d[0], a1 = d[1], a2 = d[2], a3 = d[3];
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, -%0, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %1, -%1, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %2, -%2, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %3, -%3, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
                 : "v"(c), "i"(K));
    d[0] = a0;
    d[1] = a1;
    d[2] = a2;
    d[3] = a3;
}

template <int K, bool FWD>
__device__ __forceinline__ void diag_solve_steps(d4 &d, const double (&c)[16])
{
    if constexpr (K == (FWD ? 0 : 15)) {
#pragma unroll
        for (int r = 0; r < 4; ++r) d[r] = __builtin_fma(-row_bcast<K>(d[r]), c[K], d[r]);
    } else {
        diag_step_dpp<K>(d, c[K]);
    }
    if constexpr (FWD && K < 15) diag_solve_steps<K + 1, FWD>(d, c);
    if constexpr (!FWD && K > 0) diag_solve_steps<K - 1, FWD>(d, c);
}

// Upper Gram tiles t = W, W + WAVES, ... of a PR-row panel (src = panel + (lane/16) S + lane%16),
// with the tile coordinates known at compile time.
// (the tile coordinates are template constants, so op[] stays in registers without indexing)
template <int NT, int W, int WAVES, int U, int TPW>
__device__ __forceinline__ void wide_gram_step(d4 (&acc)[TPW], const double (&op)[NT])
{
    constexpr int t = W + U * WAVES;
    if constexpr (t < NT * (NT + 1) / 2) {
        constexpr int I = tile_row(NT, t), J = tile_col(NT, t);
        acc[U] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], acc[U], 0, 0, 0);
    }
    if constexpr (U + 1 < TPW) wide_gram_step<NT, W, WAVES, U + 1, TPW>(acc, op);
}

template <int NP, int W, int WAVES, int TPW, int PR, int S>
__device__ __forceinline__ void wide_gram(d4 (&acc)[TPW], const double *src)
{
    constexpr int NT = NP / 16;
    for (int s4 = 0; s4 < PR / 4; ++s4) {
        const double *row = src + 4 * s4 * S;
        double op[NT];
#pragma unroll
        for (int b = 0; b < NT; ++b) op[b] = row[16 * b];
        wide_gram_step<NT, W, WAVES, 0, TPW>(acc, op);
    }
}

// Second operand of MODE 4 (first half of the n = 256 block solve): after the panel's
// Q_1 = X_1 R~_11^{-1} is solved, X'_2 = X_2 - Q_1 R~_12 is formed for the same rows.
struct WideProd {
    const double *X2;  // m x n2, leading dimension ldx2
    int64_t ldx2;
    double *O2;        // m x n2 result (may alias X2)
    int64_t ldo2;
    const double *R12; // 128 x n2, leading dimension ldr
    int64_t ldr;
    int n2;            // 1 .. 128
};

template <int NP, int MODE, bool VEC, bool NTC = false>
__device__ __forceinline__ void
pass_wide_body(const Problem &p, double *__restrict__ Qout, const double *__restrict__ Rt,
               const double *__restrict__ dinv, double *__restrict__ part_out,
               const Ctl *__restrict__ ctl, int pass, int final_gram, int64_t p0, int64_t p1,
               const WideProd &pr = WideProd{})
{
    constexpr int WAVES = 4;
    constexpr int PR = 64;
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int TPW = (T + WAVES - 1) / WAVES;
    constexpr int NOFF = NT * (NT - 1) / 2;
    constexpr int S = NP + 2;
    constexpr int PP = PR * NP / 2 / (WAVES * 64);  // double pairs per thread per panel
    __shared__ __attribute__((aligned(16))) double P[PR * S];
    __shared__ double bl[NOFF * 4 * 64];
    __shared__ double dtab[NT * 256 + NP];

    if (!gate(ctl, pass)) return;
    const bool want_gram = MODE == 1 && gram_needed(ctl, pass, final_gram);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int n = p.n;

    for (int idx = threadIdx.x; idx < NOFF * 4 * 64; idx += WAVES * 64) {
        const int l = idx & 63, s4 = (idx >> 6) & 3, pi = idx >> 8;
        int J = 1, K = pi;
        while (K >= J) {
            K -= J;
            ++J;
        }
        const int e = MODE == 3 ? (16 * K + (l & 15)) * NP + 16 * J + 4 * s4 + (l >> 4)
                                : (16 * K + 4 * s4 + (l >> 4)) * NP + 16 * J + (l & 15);
        bl[idx] = -as_cview(Rt)[e];
    }
    // Diagonal-block coefficients, entry (J, k, j): forward r_kj / r_kk for k < j, transposed
    // (MODE 3) r_jk / r_kk for j < k, zero elsewhere; then the reciprocal diagonal.
    for (int idx = threadIdx.x; idx < NT * 256; idx += WAVES * 64) {
        const int J = idx >> 8, k = (idx >> 4) & 15, j = idx & 15;
        double v = 0.0;
        if (MODE == 3 ? j < k : k < j) {
            const int e = MODE == 3 ? (16 * J + j) * NP + 16 * J + k : (16 * J + k) * NP + 16 * J + j;
            v = as_cview(Rt)[e] * as_cview(dinv)[16 * J + k];
        }
        dtab[idx] = v;
    }
    for (int i = threadIdx.x; i < NP; i += WAVES * 64) dtab[NT * 256 + i] = as_cview(dinv)[i];

    d4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};

    // MODE 4: -R~_12 slice of this wave in the B-operand layout, bf[cb][s4] = -R~_12[4 s4 + lk][c]
    // with c = 32 wv + 16 cb + li; the panel's X_2 in the MFMA result layout
    constexpr bool PROD = MODE == 4;
    constexpr int PC = PROD ? 2 : 1, PK = PROD ? NP / 4 : 1;
    double bf[PC][PK];
    d4 x2[PROD ? PR / 16 : 1][PC];
    const bool wprod = PROD && 32 * wv < pr.n2;
    if constexpr (PROD) {
#pragma unroll
        for (int cb = 0; cb < PC; ++cb) {
            const int c = 32 * wv + 16 * cb + li;
#pragma unroll
            for (int s4 = 0; s4 < PK; ++s4)
                bf[cb][s4] = c < pr.n2 ? -as_global(pr.R12)[(int64_t)(4 * s4 + lk) * pr.ldr + c] : 0.0;
        }
    }
    auto load_x2 = [&](int64_t pnl) {
        if constexpr (PROD) {
#pragma unroll
            for (int g = 0; g < PR / 16; ++g)
#pragma unroll
                for (int cb = 0; cb < PC; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = pnl * PR + 16 * g + lk + 4 * r;
                        const int c = 32 * wv + 16 * cb + li;
                        x2[g][cb][r] = (wprod && row < p.m && c < pr.n2) ? as_global(pr.X2)[row * pr.ldx2 + c] : 0.0;
                    }
        }
    };

    double2 pre[PP];
    auto load_panel = [&](int64_t pnl) {
        const int64_t rb = pnl * PR;
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = threadIdx.x + WAVES * 64 * i;
            const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
            const int64_t row = rb + r;
            if (VEC) {
                // buffer loads: rows past the end of the matrix read zeros, padding columns use an
                // offset outside the resource (zeros as well)
                const __amdgpu_buffer_rsrc_t rs = rows_rsrc(p.X, p.ldx, rb, p.m, n);
                const uint32_t off = c < n ? (uint32_t)((r * p.ldx + c) * 8) : kBufOut;
                pre[i] = buf_load2<NTC ? kBufStream : 0>(rs, off);
                (void)row;
            } else {
                double a = 0.0, b = 0.0;
                if (row < p.m) {
                    const gview<const double> src = as_global(p.X) + row * p.ldx + c;
                    if (c < n) a = src[0];
                    if (c + 1 < n) b = src[1];
                }
                pre[i] = make_double2(a, b);
            }
        }
    };
    if (p0 < p1) load_panel(p0);
    for (int64_t pn = p0; pn < p1; ++pn) {
        const int64_t r0 = pn * PR;
        lds_barrier();  // the previous panel is no longer read
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = threadIdx.x + WAVES * 64 * i;
            const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
            *reinterpret_cast<double2 *>(P + r * S + c) = pre[i];
        }
        lds_barrier();
        load_x2(pn);
        if (pn + 1 < p1) load_panel(pn + 1);

        // ---- substitution of rows 16 wv .. 16 wv + 15, block by block: the block's MFMA update
        // from the solved blocks, then the diagonal solve in the result layout
        const int R0 = 16 * wv;
        if constexpr (MODE == 1 || MODE == 2) {
            // (MODE 4 keeps the block-by-block order: its -R~_12 slice leaves no registers for
            // the eight blocks.)  Right-looking: every block T_J of the wave's rows stays in registers (the MFMA
            // result layout); once block K is solved, its product with -R~_KJ is added to each
            // later T_J.  Each T_J still receives X_J - Q_0 R~_0J - Q_1 R~_1J - ... in the order
            // K = 0, 1, ... (and k-steps s4 = 0..3), as in the block-by-block order, but the
            // updates of different J are independent MFMA chains.
            d4 tb[NT];
#pragma unroll
            for (int J = 0; J < NT; ++J)
#pragma unroll
                for (int r = 0; r < 4; ++r) tb[J][r] = P[(R0 + lk + 4 * r) * S + 16 * J + li];
            const double *arow = P + (R0 + li) * S + lk;
            // solve block K and store Q_K for the A operands of the updates
            auto solve_store = [&](d4 &t, int K) {
                double cf[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) cf[k] = dtab[(K * 16 + k) * 16 + li];
                const double dj = dtab[NT * 256 + 16 * K + li];
                diag_solve_steps<0, true>(t, cf);
#pragma unroll
                for (int r = 0; r < 4; ++r) P[(R0 + lk + 4 * r) * S + 16 * K + li] = t[r] * dj;
            };
            auto update = [&](d4 &t, int K, int J) {
                const int pi = J * (J - 1) / 2 + K;
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    t = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * K + 4 * s4], bl[(pi * 4 + s4) * 64 + lane], t, 0,
                                                             0, 0);
            };
            solve_store(tb[0], 0);
            wave_sync();
#pragma unroll
            for (int K = 0; K + 1 < NT; ++K) {
                // T_{K+1} is complete after Q_K's update; the updates of the later blocks by Q_K
                // do not depend on its solve
                update(tb[K + 1], K, K + 1);
#pragma unroll
                for (int J = K + 2; J < NT; ++J) update(tb[J], K, J);
                solve_store(tb[K + 1], K + 1);
                wave_sync();
            }
        } else
#pragma unroll
        for (int it = 0; it < NT; ++it) {
            const int J = MODE == 3 ? NT - 1 - it : it;
            double *blk = P + (R0 + lk) * S + 16 * J + li;
            double cf[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) cf[k] = dtab[(J * 16 + k) * 16 + li];
            const double dj = dtab[NT * 256 + 16 * J + li];
            d4 d;
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] = blk[4 * r * S];
            const double *arow = P + (R0 + li) * S + lk;
            if constexpr (MODE == 3) {
                //   T_J = Y_J - sum_{K>J} X_K R~_JK^T
#pragma unroll
                for (int J2 = J + 1; J2 < NT; ++J2) {
                    const int pi = J2 * (J2 - 1) / 2 + J;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4)
                        d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * J2 + 4 * s4], bl[(pi * 4 + s4) * 64 + lane], d,
                                                                 0, 0, 0);
                }
                diag_solve_steps<15, false>(d, cf);
            } else {
                //   T_J = X_J - sum_{K<J} Q_K R~_KJ
                const int pi0 = J * (J - 1) / 2;
#pragma unroll
                for (int K = 0; K < J; ++K)
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4)
                        d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * K + 4 * s4], bl[((pi0 + K) * 4 + s4) * 64 + lane],
                                                                 d, 0, 0, 0);
                diag_solve_steps<0, true>(d, cf);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) blk[4 * r * S] = d[r] * dj;
            wave_sync();
        }
        lds_barrier();

        // ---- Q panel -> HBM
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = threadIdx.x + WAVES * 64 * i;
            const int r = e2 / (NP / 2), c = 2 * (e2 % (NP / 2));
            const int64_t row = r0 + r;
            if constexpr (VEC) {
                // buffer stores: rows past the end and padding columns are dropped
                const __amdgpu_buffer_rsrc_t rq = rows_rsrc(Qout, p.ldq, r0, p.m, n);
                const uint32_t off = c < n ? (uint32_t)((r * p.ldq + c) * 8) : kBufOut;
                buf_store2<NTC ? kBufStream : 0>(rq, off, *reinterpret_cast<const double2 *>(P + r * S + c));
            } else if (row < p.m && c < n) {
                const double2 v = *reinterpret_cast<const double2 *>(P + r * S + c);
                const gview<double> dst = as_global(Qout) + row * p.ldq + c;
                dst[0] = v.x;
                if (c + 1 < n) dst[1] = v.y;
            }
        }

        // ---- MODE 4: X'_2 = X_2 - Q_1 R~_12 for the panel (Q_1 in LDS, all waves' strips solved)
        if (wprod) {
            const double *abase = P + li * S + lk;
#pragma unroll
            for (int g = 0; g < PR / 16; ++g) {
#pragma unroll
                for (int cb = 0; cb < PC; ++cb) {
                    d4 d = x2[g][cb];
                    const double *arow = abase + 16 * g * S;
#pragma unroll
                    for (int s4 = 0; s4 < PK; ++s4)
                        d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[4 * s4], bf[cb][s4], d, 0, 0, 0);
                    const int c = 32 * wv + 16 * cb + li;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = r0 + 16 * g + lk + 4 * r;
                        if (row < p.m && c < pr.n2) as_global(pr.O2)[row * pr.ldo2 + c] = d[r];
                    }
                }
            }
        }

        // ---- Gram tiles of this wave over the 64 rows
        if (want_gram) {
            const double *src = P + lk * S + li;
            switch (wv) {
            case 0: wide_gram<NP, 0, WAVES, TPW, PR, S>(acc, src); break;
            case 1: wide_gram<NP, 1, WAVES, TPW, PR, S>(acc, src); break;
            case 2: wide_gram<NP, 2, WAVES, TPW, PR, S>(acc, src); break;
            default: wide_gram<NP, 3, WAVES, TPW, PR, S>(acc, src); break;
            }
        }
    }
    if (!want_gram) return;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wv + u * WAVES;
        if (t < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) part_out[t * 256 + r * 64 + lane] = acc[u][r];
        }
    }
}

template <int NP, int MODE, bool VEC>
__global__ void __launch_bounds__(256)
k_pass_wide(Problem p, double *__restrict__ Qout, const double *__restrict__ Rt,
            const double *__restrict__ dinv, double *__restrict__ partials,
            const Ctl *__restrict__ ctl, int pass, int final_gram)
{
    constexpr int NT = NP / 16;
    constexpr int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    const int64_t npanels = (p.m + 63) / 64;
    const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    // one problem: X and Q are streamed once per pass (non-temporal accesses)
    pass_wide_body<NP, MODE, VEC, true>(p, Qout, Rt, dinv, partials + (int64_t)blockIdx.x * E, ctl, pass,
                                        final_gram, p0 < p1 ? p0 : p1, p1);
}

// MODE 4 (NP = 128): the first half of the n = 256 block solve with the product for the second.
template <bool VEC>
__global__ void __launch_bounds__(256)
k_pass_wide4(Problem p, double *__restrict__ Qout, const double *__restrict__ Rt,
             const double *__restrict__ dinv, WideProd pr, const Ctl *__restrict__ ctl, int pass)
{
    const int64_t npanels = (p.m + 63) / 64;
    const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    pass_wide_body<128, 4, VEC, true>(p, Qout, Rt, dinv, nullptr, ctl, pass, 0, p0 < p1 ? p0 : p1, p1, pr);
}


template <int NP, int MODE, bool VEC>
__global__ void __launch_bounds__(256)
k_pass_wide_b(const BatchInst *__restrict__ insts, const BatchTask *__restrict__ tasks,
              double *__restrict__ partials, int pass, int final_gram)
{
    constexpr int NT = NP / 16;
    constexpr int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    const BatchTask t = load_cview(tasks + blockIdx.x);
    const BatchInst I = load_cview(insts + t.inst);
    Problem p = I.p;
    if (pass > 1) {
        p.X = p.Q;
        p.ldx = p.ldq;
    }
    pass_wide_body<NP, MODE, VEC, true>(p, p.Q, factor_of(I.w, NP, pass), dinv_of(I.w, NP, pass),
                                  partials + (int64_t)blockIdx.x * E, I.w.ctl, pass, final_gram, t.r0 / 64,
                                  (t.r1 + 63) / 64);
}

// Threads of the Gram kernel: 16 waves at n = 256 (9 of the 136 tiles per wave, 128 registers:
// four waves per SIMD; 8 waves for the binary32 variant, whose extra accumulators would spill),
// 8 waves for the first-pass B-Gram at n >= 64 (its two sets of tile accumulators, X^T B X and
// X^T X, then fit two waves per SIMD) and for the Euclidean Gram at n = 128 (5 of the 36 tiles per
// wave, 116 registers: two workgroups, four waves per SIMD; 10^6 x 128 4.12 -> 4.06 ms, the c4
// batch 61.3 -> 59.1 ms), 4 waves otherwise (measured faster for the B-Gram alone: two 4-wave
// workgroups per CU).
constexpr int gram_wide_threads(int np, bool obl, bool euc, bool f32)
{
    return np == 256 ? (f32 ? 512 : 1024) : ((obl && euc && np >= 64) || (np == 128 && !obl && !f32) ? 512 : 256);
}

// ------------------------------------------------------------------------------------------
// Gram for n <= 256 with panels of 64 rows (32 with B, 16 at n = 256) shared by the waves of the
// workgroup (gram_wide_threads): wave w owns the upper tiles t = w, w + WV, ...; its operands are
// read from LDS at wave-uniform tile offsets.  The next panel's loads are issued before the
// current panel's MFMAs.
//   OBL: B-Gram X^T (B X), B tridiagonal: the panel carries one halo row above and below and
//        Y = B X is formed once per panel in LDS, (B x)_k = off_{k-1} x_{k-1} + diag_k x_k +
//        off_k x_{k+1}.
//   EUC: with OBL, also X^T X (second half of the partial) and the workgroup's Gershgorin
//        maximum of B (for the first-pass shift of equation (eq:finds2B)).
//   F32: binary32 MFMA over each panel (64 rows; 16 for n = 256), added to the binary64 tiles
//        after the panel.
//   BATCH: workgroup b takes task b of the device task table; otherwise workgroup b takes a
//        contiguous share of the problem's panels.
template <int NP, bool OBL, bool EUC, bool F32, bool BATCH>
__global__ void __launch_bounds__(gram_wide_threads(NP, OBL, EUC, F32))
k_gram_wide(Problem p, double *__restrict__ partials, double *__restrict__ bmax,
            const Ctl *__restrict__ ctl, int pass, int final_gram,
            const BatchInst *__restrict__ insts, const BatchTask *__restrict__ tasks)
{
    constexpr int NTH = gram_wide_threads(NP, OBL, EUC, F32);
    constexpr int WV = NTH / 64;  // waves
    static_assert(!(NP == 256 && OBL), "the n = 256 B-Gram uses k_gram_lds");
    // rows per panel: 32 with B (X and Y = B X both staged, two workgroups per CU), 16 at n = 256
    // (17 tile accumulators per wave leave room for a 16-row prefetch only)
    constexpr int PR = NP == 256 ? 16 : (OBL ? 32 : 64);
    constexpr int H = OBL ? 1 : 0;
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int TPW = (T + WV - 1) / WV;
    constexpr int S = lds_stride_gram(NP);
    constexpr int PP = PR * NP / 2 / NTH;  // double pairs per thread per panel
    static_assert(PP >= 1 && (PR * NP / 2) % NTH == 0, "panel must split over the workgroup");
    static_assert(!F32 || PR == f32_chain_rows(NP), "a binary32 chain is one panel");
    constexpr int64_t E = (int64_t)T * 256;
    __shared__ __attribute__((aligned(16))) double xs[(PR + 2 * H) * S];
    __shared__ __attribute__((aligned(16))) double ys[OBL ? PR * S : 1];
    __shared__ double cs[OBL ? 3 * PR : 1];
    __shared__ double gm[EUC ? NTH : 1];

    int64_t p0, p1;
    if constexpr (BATCH) {
        const BatchTask tk = load_cview(tasks + blockIdx.x);
        const BatchInst I = load_cview(insts + tk.inst);
        p = I.p;
        if (pass >= 1) {  // the Gram of pass >= 1 reads the Q its substitution just wrote
            p.X = p.Q;
            p.ldx = p.ldq;
        }
        ctl = I.w.ctl;
        p0 = tk.r0 / PR;
        p1 = (tk.r1 + PR - 1) / PR;
    } else {
        const int64_t npanels = (p.m + PR - 1) / PR;
        const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
        p0 = (int64_t)blockIdx.x * per;
        p1 = (p0 + per < npanels) ? p0 + per : npanels;
        if (p0 > p1) p0 = p1;
    }
    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int n = p.n;

    d4 acc[TPW], acce[EUC ? TPW : 1];
    f4 a32[F32 ? TPW : 1];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < (EUC ? TPW : 1); ++u) acce[u] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < (F32 ? TPW : 1); ++u) a32[u] = (f4){0.f, 0.f, 0.f, 0.f};
    double bm = 0.0;
    // column offsets (16 I, 16 J) of this wave's tiles t = wv + 4u
    int ti[TPW], tj[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        int I = 0, J = 0;
        tile_ij(NT, wv + WV * u < T ? wv + WV * u : 0, I, J);
        ti[u] = 16 * I;
        tj[u] = 16 * J;
    }

    double2 pre[PP], hal = make_double2(0.0, 0.0);
    double clo = 0.0, cd = 0.0, cup = 0.0;
    auto pair_at = [&](int64_t row, int c) -> double2 {
        double a = 0.0, b = 0.0;
        if (row >= 0 && row < p.m) {
            const gview<const double> src = as_global(p.X) + row * p.ldx + c;
            if (c < n) a = src[0];
            if (c + 1 < n) b = src[1];
        }
        return make_double2(a, b);
    };
    auto load_panel = [&](int64_t pnl) {
        const int64_t rb = pnl * PR;
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + NTH * i;
            pre[i] = pair_at(rb + e2 / (NP / 2), 2 * (e2 % (NP / 2)));
        }
        if (OBL) {
            if (t < NP) {  // halo rows rb - 1 (t < NP/2) and rb + PR
                const int hr = t / (NP / 2), c = 2 * (t % (NP / 2));
                hal = pair_at(hr == 0 ? rb - 1 : rb + PR, c);
            }
            if (t < PR) {
                const int64_t row = rb + t;
                clo = cd = cup = 0.0;
                if (row < p.m) {
                    cd = as_global(p.bdiag)[row];
                    if (row > 0) clo = as_global(p.boff)[row - 1];
                    if (row + 1 < p.m) cup = as_global(p.boff)[row];
                }
            }
        }
    };
    if (p0 < p1) load_panel(p0);
    for (int64_t pn = p0; pn < p1; ++pn) {
        __syncthreads();  // the previous panel is no longer read
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + NTH * i;
            *reinterpret_cast<double2 *>(xs + (H + e2 / (NP / 2)) * S + 2 * (e2 % (NP / 2))) = pre[i];
        }
        if (OBL) {
            if (t < NP) {
                const int hr = t / (NP / 2), c = 2 * (t % (NP / 2));
                *reinterpret_cast<double2 *>(xs + (hr == 0 ? 0 : PR + 1) * S + c) = hal;
            }
            if (t < PR) {
                cs[3 * t] = clo;
                cs[3 * t + 1] = cd;
                cs[3 * t + 2] = cup;
                if (EUC && pn * PR + t < p.m) {
                    double g = fabs(clo) + fabs(cd);
                    g = g + fabs(cup);
                    bm = g > bm ? g : bm;
                }
            }
        }
        __syncthreads();
        if (pn + 1 < p1) load_panel(pn + 1);
        if (OBL) {
            // Y = B X for the 64 panel rows
#pragma unroll
            for (int i = 0; i < PR * NP / NTH; ++i) {
                const int e = t + NTH * i;
                const int r = e / NP, c = e % NP;
                const double *xc = xs + (r + 1) * S + c;
                const double bx = cs[3 * r] * xc[-S] + cs[3 * r + 1] * xc[0];
                ys[r * S + c] = bx + cs[3 * r + 2] * xc[S];
            }
            __syncthreads();
        }
        const double *xsrc = xs + (H + (lane >> 4)) * S + (lane & 15);
        const double *ysrc = OBL ? ys + (lane >> 4) * S + (lane & 15) : xsrc;
#pragma unroll 2
        for (int s4 = 0; s4 < PR / 4; ++s4) {
            const double *xr = xsrc + 4 * s4 * S;
            const double *yr = ysrc + 4 * s4 * S;
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                if (wv + WV * u < T) {
                    const double a = xr[ti[u]];
                    const double b = yr[tj[u]];
                    if (F32)
                        a32[F32 ? u : 0] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, a32[F32 ? u : 0], 0, 0, 0);
                    else
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
                    if (EUC)
                        acce[EUC ? u : 0] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(a, xr[tj[u]], acce[EUC ? u : 0], 0, 0, 0);
                }
            }
        }
        if (F32) {
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[u][r] += (double)a32[F32 ? u : 0][r];
                a32[F32 ? u : 0] = (f4){0.f, 0.f, 0.f, 0.f};
            }
        }
    }
    double *out = partials + (int64_t)blockIdx.x * (EUC ? 2 * E : E);
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int tt = wv + u * WV;
        if (tt < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                out[tt * 256 + r * 64 + lane] = acc[u][r];
                if (EUC) out[E + tt * 256 + r * 64 + lane] = acce[EUC ? u : 0][r];
            }
        }
    }
    if (EUC) {
        gm[t] = bm;
        __syncthreads();
        if (t == 0) {
            double g = 0.0;
            for (int i = 0; i < NTH; ++i) g = gm[i] > g ? gm[i] : g;
            bmax[blockIdx.x] = g;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Tall-skinny product with a small right factor on FP64 MFMA:
//   Out[:, c0 + j] = Base[:, c0 + j] + SIGN * sum_{k < K} A[:, k] B[k, c0 + j],  j < NB,
// over column blocks of NB columns (columns at or beyond ncols are not written).  The grid is
// (panel groups) x (column blocks); when the number of groups is a multiple of 8 the dispatch
// order is remapped so that the column blocks of one panel group are consecutive workgroups of
// one XCD (dispatch goes round-robin over the 8 XCDs): they run together and share the XCD's L2
// for A, which HBM then delivers once instead of once per column block.  The workgroup stages
// its K x NB block of B once in LDS in the MFMA B-operand layout (TRANS: B is read transposed,
// B[k][j] = Bm[j][k]) and streams 32-row panels of A through LDS, the next panel's loads issued
// before the current panel's MFMAs.  Wave w owns the 16x16 output tiles
// t = w, w + 4, ... of a panel (2 row groups x NB/16 column groups); its Base elements are
// loaded with the panel, one panel ahead.  Base may equal Out (each element is read by the lane
// that writes it, before the write, and panels are disjoint); A must not overlap Out.  Predicated on
// the control block like the pass kernels (gate), and with min_pass > 0 on at least min_pass
// passes having been applied.
template <int K, int NB, bool TRANS, int SIGN>
__global__ void __launch_bounds__(256)
k_mm(int64_t m, int ncols, int ka, const double *__restrict__ A, int64_t lda, const double *__restrict__ Bm,
     int64_t ldb, const double *Base, int64_t ldbase, double *Out, int64_t ldo, const Ctl *__restrict__ ctl,
     int pass, int min_pass)
{
    constexpr int PR = 32;
    constexpr int SA = K + 2;
    constexpr int KS = K / 4;          // MFMA k-steps
    constexpr int CB = NB / 16;        // column groups
    constexpr int TILES = 2 * CB;      // output tiles per panel
    constexpr int TPW = (TILES + 3) / 4;
    constexpr int PP = PR * K / 2 / 256;  // A pairs per thread per panel
    static_assert(PP >= 1 && (PR * K / 2) % 256 == 0, "panel must split over the workgroup");
    __shared__ __attribute__((aligned(16))) double as[PR * SA];
    __shared__ double bs[KS * CB * 64];
    if (!gate(ctl, pass)) return;
    if (min_pass > 0 && ctl->pass < min_pass) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ngrp = gridDim.x, ncb = gridDim.y;
    int grp = blockIdx.x, cb = blockIdx.y;
    if ((ngrp & 7) == 0) {
        const int b = blockIdx.x + ngrp * blockIdx.y, j = b >> 3;
        cb = j % ncb;
        grp = (j / ncb) * 8 + (b & 7);
    }
    const int c0 = NB * cb;

    // B block in the B-operand layout: entry (s, cg, l) = B[4 s + l / 16][c0 + 16 cg + l % 16]
    for (int idx = t; idx < KS * CB * 64; idx += 256) {
        const int l = idx & 63, cg = (idx >> 6) % CB, s4 = idx / (64 * CB);
        const int k = 4 * s4 + (l >> 4), j = c0 + 16 * cg + (l & 15);
        double v = 0.0;
        if (k < ka && j < ncols) v = TRANS ? as_cview(Bm)[(int64_t)j * ldb + k] : as_cview(Bm)[(int64_t)k * ldb + j];
        bs[idx] = v;
    }

    const int64_t npanels = (m + PR - 1) / PR;
    const int64_t per = (npanels + ngrp - 1) / ngrp;
    int64_t p0 = (int64_t)grp * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    if (p0 > p1) p0 = p1;

    // tiles of this wave: row group rg, column group cg
    int trg[TPW], tcg[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int tt = wv + 4 * u;
        trg[u] = tt < TILES ? tt / CB : 0;
        tcg[u] = tt < TILES ? tt % CB : 0;
    }
    // A panel pairs and the wave's Base elements of a panel, loaded one panel ahead
    double2 pre[PP];
    double bpre[TPW][4];
    auto load_panel = [&](int64_t pnl) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + 256 * i;
            const int r = e2 / (K / 2), c = 2 * (e2 % (K / 2));
            const int64_t row = pnl * PR + r;
            double a = 0.0, b = 0.0;
            if (row < m) {
                const gview<const double> src = as_global(A) + row * lda + c;
                if (c < ka) a = src[0];
                if (c + 1 < ka) b = src[1];
            }
            pre[i] = make_double2(a, b);
        }
#pragma unroll
        for (int u = 0; u < TPW; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = pnl * PR + 16 * trg[u] + (lane >> 4) + 4 * r;
                const int col = c0 + 16 * tcg[u] + (lane & 15);
                double b0 = 0.0;
                if (Base && wv + 4 * u < TILES && row < m && col < ncols) b0 = as_global(Base)[row * ldbase + col];
                bpre[u][r] = b0;
            }
    };
    if (p0 < p1) load_panel(p0);
    for (int64_t pn = p0; pn < p1; ++pn) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + 256 * i;
            *reinterpret_cast<double2 *>(as + (e2 / (K / 2)) * SA + 2 * (e2 % (K / 2))) = pre[i];
        }
        double bcur[TPW][4];
#pragma unroll
        for (int u = 0; u < TPW; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) bcur[u][r] = bpre[u][r];
        __syncthreads();
        if (pn + 1 < p1) load_panel(pn + 1);
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (wv + 4 * u >= TILES) continue;
            d4 d = (d4){0.0, 0.0, 0.0, 0.0};
            const double *arow = as + (16 * trg[u] + (lane & 15)) * SA + (lane >> 4);
            const double *bcol = bs + tcg[u] * 64 + lane;
#pragma unroll 8
            for (int s4 = 0; s4 < KS; ++s4)
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[4 * s4], bcol[s4 * CB * 64], d, 0, 0, 0);
            // element (i, j) = (lane / 16 + 4 r, lane % 16) of the tile
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = pn * PR + 16 * trg[u] + (lane >> 4) + 4 * r;
                const int col = c0 + 16 * tcg[u] + (lane & 15);
                if (row < m && col < ncols) as_global(Out)[row * ldo + col] = SIGN > 0 ? bcur[u][r] + d[r] : bcur[u][r] - d[r];
            }
        }
    }
}

// The same product for K = 128 / 256 with the right factor in registers: the workgroup owns a
// 64-column block, wave w the 16 columns c0 + 16 w .. c0 + 16 w + 15, whose K x 16 slice of B it
// keeps in registers in the MFMA B-operand layout (loaded once).  Panels of A (32 rows; 16 at
// K = 256, which keeps the wave within 256 registers, two waves per SIMD) are staged in LDS one
// panel ahead as in k_mm, and each wave computes the panel's 16-row tiles of its columns: one
// LDS operand read per MFMA and one accumulation chain per tile.  Dispatch order, Base and
// predication as in k_mm.
template <int K, bool TRANS, int SIGN>
__global__ void __launch_bounds__(256)
k_mm_breg(int64_t m, int ncols, int ka, const double *__restrict__ A, int64_t lda, const double *__restrict__ Bm,
          int64_t ldb, const double *Base, int64_t ldbase, double *Out, int64_t ldo, const Ctl *__restrict__ ctl,
          int pass, int min_pass)
{
    constexpr int PR = K == 256 ? 16 : 32;
    constexpr int RG = PR / 16;
    constexpr int SA = K + 2;
    constexpr int KS = K / 4;
    constexpr int NB = 64;
    constexpr int PP = PR * K / 2 / 256;
    static_assert(K == 128 || K == 256, "k_mm_breg serves K = 128 and 256");
    __shared__ __attribute__((aligned(16))) double as[PR * SA];
    if (!gate(ctl, pass)) return;
    if (min_pass > 0 && ctl->pass < min_pass) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ngrp = gridDim.x, ncb = gridDim.y;
    int grp = blockIdx.x, cb = blockIdx.y;
    if ((ngrp & 7) == 0) {
        const int b = blockIdx.x + ngrp * blockIdx.y, j = b >> 3;
        cb = j % ncb;
        grp = (j / ncb) * 8 + (b & 7);
    }
    const int col = NB * cb + 16 * wv + (lane & 15);
    const bool colok = col < ncols;

    // B slice: bf[s4] = B[4 s4 + lane / 16][col]
    double bf[KS];
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4) {
        const int k = 4 * s4 + (lane >> 4);
        double v = 0.0;
        if (colok && k < ka) v = TRANS ? as_global(Bm)[(int64_t)col * ldb + k] : as_global(Bm)[(int64_t)k * ldb + col];
        bf[s4] = v;
    }

    const int64_t npanels = (m + PR - 1) / PR;
    const int64_t per = (npanels + ngrp - 1) / ngrp;
    int64_t p0 = (int64_t)grp * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    if (p0 > p1) p0 = p1;

    double2 pre[PP];
    double bpre[RG][4];
    auto load_panel = [&](int64_t pnl) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + 256 * i;
            const int r = e2 / (K / 2), c = 2 * (e2 % (K / 2));
            const int64_t row = pnl * PR + r;
            double a = 0.0, b = 0.0;
            if (row < m) {
                const gview<const double> src = as_global(A) + row * lda + c;
                if (c < ka) a = src[0];
                if (c + 1 < ka) b = src[1];
            }
            pre[i] = make_double2(a, b);
        }
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = pnl * PR + 16 * g + (lane >> 4) + 4 * r;
                double b0 = 0.0;
                if (Base && colok && row < m) b0 = as_global(Base)[row * ldbase + col];
                bpre[g][r] = b0;
            }
    };
    if (p0 < p1) load_panel(p0);
    for (int64_t pn = p0; pn < p1; ++pn) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int e2 = t + 256 * i;
            *reinterpret_cast<double2 *>(as + (e2 / (K / 2)) * SA + 2 * (e2 % (K / 2))) = pre[i];
        }
        double bcur[RG][4];
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) bcur[g][r] = bpre[g][r];
        __syncthreads();
        if (pn + 1 < p1) load_panel(pn + 1);

        d4 acc[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[g] = (d4){0.0, 0.0, 0.0, 0.0};
        const double *a0 = as + (lane & 15) * SA + (lane >> 4);
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
#pragma unroll
            for (int g = 0; g < RG; ++g)
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[16 * g * SA + 4 * s4], bf[s4], acc[g], 0, 0, 0);
        }
        // element (i, j) = (lane / 16 + 4 r, lane % 16) of tile g
        if (colok) {
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = pn * PR + 16 * g + (lane >> 4) + 4 * r;
                    if (row < m) as_global(Out)[row * ldo + col] = SIGN > 0 ? bcur[g][r] + acc[g][r] : bcur[g][r] - acc[g][r];
                }
        }
    }
}

// The diagonal 128 x 128 blocks of a 256-wide factor (identity padding kept) and their
// reciprocal diagonals, copied to the stride-128 slots the 128-wide substitution reads:
// Rsplit = [R~_11 | R~_22 | 1/diag(R~_11) | 1/diag(R~_22)].
__global__ void __launch_bounds__(256)
k_split256(const double *__restrict__ Rt, const double *__restrict__ dinv, double *__restrict__ Rsplit,
           const Ctl *__restrict__ ctl, int pass)
{
    if (!gate(ctl, pass)) return;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < 2 * 128 * 128; e += gridDim.x * 256) {
        const int b = e >> 14, i = (e >> 7) & 127, j = e & 127;
        Rsplit[e] = Rt[(128 * b + i) * 256 + 128 * b + j];
    }
    if (blockIdx.x == 0) Rsplit[2 * 128 * 128 + threadIdx.x] = dinv[threadIdx.x];
}

// ------------------------------------------------------------------------------------------
// Row-wise substitution of the batched n = 256 class, one row per thread, 64-column blocks: block J starts from
// x_J, receives -q_k r_kj for every earlier k in increasing order (solved values are re-read
// from the thread's own output row), then is solved against the diagonal block.
template <int NP>
__device__ __forceinline__ void
trsm_big_body(const Problem &p, const double *__restrict__ Rt, const double *__restrict__ dinv,
              const Ctl *__restrict__ ctl, int pass, int64_t row0, int64_t rstride, int64_t rend)
{
    if (!gate(ctl, pass)) return;
    const int n = p.n;
    for (int64_t row = row0 + threadIdx.x; row < rend; row += rstride) {
        const gview<const double> xr = as_global(p.X) + row * p.ldx;
        const gview<double> qr = as_global(p.Q) + row * p.ldq;
        for (int J = 0; J < NP / 64; ++J) {
            double t[64];
#pragma unroll
            for (int c = 0; c < 64; ++c) t[c] = (64 * J + c < n) ? xr[64 * J + c] : 0.0;
            for (int K = 0; K < J; ++K) {
                for (int kk = 0; kk < 64; ++kk) {
                    const int k = 64 * K + kk;
                    const double qk = (k < n) ? qr[k] : 0.0;
                    const cview<double> rk = as_cview(Rt) + (int64_t)k * NP + 64 * J;
#pragma unroll
                    for (int c = 0; c < 64; ++c) t[c] = __builtin_fma(-qk, rk[c], t[c]);
                }
            }
            const cview<double> rd = as_cview(Rt) + (int64_t)(64 * J) * NP + 64 * J;
#pragma unroll
            for (int k = 0; k < 64; ++k) {
                const double qk = t[k] * as_cview(dinv)[64 * J + k];
                t[k] = qk;
#pragma unroll
                for (int j = k + 1; j < 64; ++j) t[j] = __builtin_fma(-qk, rd[k * NP + j], t[j]);
            }
#pragma unroll
            for (int c = 0; c < 64; ++c)
                if (64 * J + c < n) qr[64 * J + c] = t[c];
        }
    }
}

template <int NP>
__global__ void __launch_bounds__(256)
k_trsm_big_b(const BatchInst *__restrict__ insts, const BatchTask *__restrict__ tasks, int pass)
{
    const BatchTask t = load_cview(tasks + blockIdx.x);
    const BatchInst I = load_cview(insts + t.inst);
    Problem p = I.p;
    if (pass > 1) {
        p.X = p.Q;
        p.ldx = p.ldq;
    }
    trsm_big_body<NP>(p, factor_of(I.w, NP, pass), dinv_of(I.w, NP, pass), I.w.ctl, pass, t.r0, 256, t.r1);
}

// ------------------------------------------------------------------------------------------
// LDS-staged Gram for any NP (used for n > 64 and for the oblique inner product).  A workgroup
// of WAVES waves streams 16-row panels through LDS; wave w owns the upper tiles t with
// t % WAVES == w and accumulates them over every row of the workgroup's share.
//   OBL: B-Gram X^T (B X) with B tridiagonal; the panel carries one halo row above and below
//        and (B x)_k = off_{k-1} x_{k-1} + diag_k x_k + off_k x_{k+1} is formed on the fly.
//   EUC: with OBL, also the Euclidean X^T X (second half of the partial) and the per-workgroup
//        Gershgorin maximum of B (first-pass shift of equation (eq:finds2B)).
//   F32: binary32 MFMA, flushed to binary64 after every f32_chain_rows(NP) rows.
//   The workgroup takes the 16-row panels [p0, p1) and writes its partial to part_out (and its
//   Gershgorin maximum to *bmax_out).
template <int NP, int WAVES, bool OBL, bool EUC, bool F32>
__device__ __forceinline__ void
gram_lds_body(const Problem &p, double *__restrict__ part_out, double *__restrict__ bmax_out,
              const Ctl *__restrict__ ctl, int pass, int final_gram, int64_t p0, int64_t p1)
{
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr int TPW = (T + WAVES - 1) / WAVES;
    constexpr int PR = 16;  // rows per panel
    constexpr int S = NP + 1;
    constexpr int HALO = OBL ? 1 : 0;
    __shared__ double xs[(PR + 2 * HALO) * S];
    __shared__ double cs[OBL ? 3 * (PR) : 1];  // off_{k-1}, diag_k, off_k of the panel rows
    __shared__ double gmax[WAVES * 64];

    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;

    const int nthr = WAVES * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = p.n;

    d4 acc[TPW], acce[EUC ? TPW : 1];
    f4 a32[F32 ? TPW : 1];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
    if (EUC) {
#pragma unroll
        for (int u = 0; u < (EUC ? TPW : 1); ++u) acce[u] = (d4){0.0, 0.0, 0.0, 0.0};
    }
    if (F32) {
#pragma unroll
        for (int u = 0; u < (F32 ? TPW : 1); ++u) a32[u] = (f4){0.f, 0.f, 0.f, 0.f};
    }
    double bm = 0.0;
    int chain = 0;
    // column offsets (16 I, 16 J) of this wave's tiles t = wv + WAVES u
    int ti[TPW], tj[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wv + u * WAVES < T ? wv + u * WAVES : 0;
        ti[u] = 16 * tile_row(NT, t);
        tj[u] = 16 * tile_col(NT, t);
    }

    for (int64_t pn = p0; pn < p1; ++pn) {
        const int64_t r0 = pn * PR;
        __syncthreads();
        for (int idx = threadIdx.x; idx < (PR + 2 * HALO) * NP; idx += nthr) {
            const int rr = idx / NP, c = idx % NP;
            const int64_t row = r0 + rr - HALO;
            double v = 0.0;
            if (row >= 0 && row < p.m && c < n) v = as_global(p.X)[row * p.ldx + c];
            xs[rr * S + c] = v;
        }
        if (OBL) {
            for (int rr = threadIdx.x; rr < PR; rr += nthr) {
                const int64_t row = r0 + rr;
                double lo = 0.0, d = 0.0, up = 0.0;
                if (row < p.m) {
                    d = as_global(p.bdiag)[row];
                    if (row > 0) lo = as_global(p.boff)[row - 1];
                    if (row + 1 < p.m) up = as_global(p.boff)[row];
                    if (EUC) {
                        double g = (row > 0 ? fabs(lo) : 0.0) + fabs(d);
                        if (row + 1 < p.m) g = g + fabs(up);
                        bm = g > bm ? g : bm;
                    }
                }
                cs[3 * rr + 0] = lo;
                cs[3 * rr + 1] = d;
                cs[3 * rr + 2] = up;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PR / 4; ++s) {
            const int rr = 4 * s + (lane >> 4);
            const double *xrow = xs + (rr + HALO) * S + (lane & 15);
            double c_lo = 0.0, c_d = 0.0, c_up = 0.0;
            if (OBL) {
                c_lo = cs[3 * rr + 0];
                c_d = cs[3 * rr + 1];
                c_up = cs[3 * rr + 2];
            }
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int t = wv + u * WAVES;
                if (t < T) {
                    const double a = xrow[ti[u]];
                    double b = xrow[tj[u]];
                    if (OBL) {
                        // (B x)_k, evaluated as off_{k-1} x_{k-1} + diag_k x_k, + off_k x_{k+1}
                        const double bx = c_lo * xrow[tj[u] - S] + c_d * b;
                        const double by = bx + c_up * xrow[tj[u] + S];
                        if (EUC) acce[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acce[u], 0, 0, 0);
                        b = by;
                    }
                    if (F32)
                        a32[F32 ? u : 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            (float)a, (float)b, a32[F32 ? u : 0], 0, 0, 0);
                    else
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
                }
            }
        }
        if (F32) {
            chain += PR;
            if (chain >= f32_chain_rows(NP) || pn + 1 == p1) {
                chain = 0;
#pragma unroll
                for (int u = 0; u < TPW; ++u) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u][r] += (double)a32[F32 ? u : 0][r];
                    a32[F32 ? u : 0] = (f4){0.f, 0.f, 0.f, 0.f};
                }
            }
        }
    }
    const int64_t E = (int64_t)T * 256;
    double *out = part_out;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wv + u * WAVES;
        if (t < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                out[t * 256 + r * 64 + lane] = acc[u][r];
                if (EUC) out[E + t * 256 + r * 64 + lane] = acce[EUC ? u : 0][r];
            }
        }
    }
    if (EUC) {
        gmax[threadIdx.x] = bm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double g = 0.0;
            for (int i = 0; i < nthr; ++i) g = gmax[i] > g ? gmax[i] : g;
            *bmax_out = g;
        }
    }
}

template <int NP, int WAVES, bool OBL, bool EUC, bool F32>
__global__ void __launch_bounds__(WAVES * 64)
k_gram_lds(Problem p, double *__restrict__ partials, double *__restrict__ bmax,
           const Ctl *__restrict__ ctl, int pass, int final_gram)
{
    constexpr int NT = NP / 16;
    constexpr int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    const int64_t npanels = (p.m + 15) / 16;
    // contiguous share of 16-row panels per workgroup
    const int64_t per = (npanels + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per;
    const int64_t p1 = (p0 + per < npanels) ? p0 + per : npanels;
    gram_lds_body<NP, WAVES, OBL, EUC, F32>(p, partials + (int64_t)blockIdx.x * (EUC ? 2 * E : E),
                                            bmax + blockIdx.x, ctl, pass, final_gram, p0, p1);
}

// ------------------------------------------------------------------------------------------
// Oblique Gram X^T B X for a general sparse B in compressed sparse rows (Section 7).  A
// workgroup takes a contiguous share of 16-row panels.  For each panel it stages the rows of X
// in LDS, stages the panel's CSR entries (row pointers, then columns and values in chunks of
// up to CSR_CHUNK entries) in LDS, and forms the matching rows of Y = B X beside X: the 16 rows
// at once, TR = NTHR / 16 threads per row, thread tc of a row taking columns tc + TR q.  Each
// output sums, in storage order, val_e x_{col_e, c} over the entries e of its row, the rows
// x_{col_e} gathered from HBM through the caches (read coalesced by the TR threads of the row;
// with the indices already in LDS, the loads of several entries are in flight together).  The
// upper tiles of X^T Y then accumulate on FP64 MFMA as in the tridiagonal kernels.  Y never
// reaches HBM: the blocked strategy of Section 7 with blocks of 16 rows of Y (all n columns)
// instead of column blocks.
//   KIND 0: X^T B X into partial slots of E = T * 256 doubles.
//   KIND 1 (first pass): also X^T X for ||X||_2 of (eq:finds2B), slots of 2 E (X^T B X, then
//   X^T X), and the Gershgorin bound (largest absolute row sum, each row summed in storage
//   order) of the workgroup's rows into bmax.
//   KIND 2 and 3 split KIND 1 over two launches where one set of tiles is all the registers
//   hold (n = 256): 2 writes X^T B X into the first half of the 2 E slots, 3 the second half
//   (X^T X, no gathers) and the Gershgorin bound.
// Row pointers outside [0, nnz] or out of order, and columns outside [0, m), are never used as
// addresses: the entries concerned are skipped and *p.bad_b set.
constexpr int CSR_CHUNK = 1024;
// Waves per SIMD the CSR Gram is compiled for (its loads wait on gathers; more waves in flight
// hide more of that latency): 5 up to n = 64, 3 at n = 128; one fewer (no spills) with both sets
// of tiles of the first pass.
constexpr int csr_min_waves(int np, int kind)
{
    return (np <= 64 ? 5 : (np == 128 ? 3 : 1)) - (kind == 1 && np >= 64 ? 1 : 0);
}

template <int NP, int WAVES, int KIND>
__global__ void __launch_bounds__(WAVES * 64, csr_min_waves(NP, KIND))
k_gram_csr(Problem p, double *__restrict__ partials, double *__restrict__ bmax, const Ctl *__restrict__ ctl,
           int pass, int final_gram)
{
    constexpr int NT = NP / 16;
    constexpr int T = NT * (NT + 1) / 2;
    constexpr bool BG = KIND != 3;                // X^T B X tiles (and the gathers for Y)
    constexpr bool EUC = KIND == 1 || KIND == 3;  // X^T X tiles and the Gershgorin bound
    // virtual tiles: with both sets, v < T is a tile of X^T B X and v >= T one of X^T X; wave w
    // takes v = w + WAVES u.  Tile v goes to slot offset VOFF + v * 256.
    constexpr int VT = (BG ? T : 0) + (EUC ? T : 0);
    constexpr int64_t SLOT = (int64_t)(KIND == 0 ? 1 : 2) * T * 256;
    constexpr int64_t VOFF = KIND == 3 ? (int64_t)T * 256 : 0;
    constexpr int TPW = (VT + WAVES - 1) / WAVES;
    constexpr int PR = 16;
    constexpr int S = NP + 1;
    constexpr int NTHR = WAVES * 64;
    constexpr int TR = NTHR / PR;      // threads per row of Y
    constexpr int CPT = NP / TR;       // columns per thread
    // entries whose loads are issued together, CPT loads each
    constexpr int GB = NP == 256 ? 1 : (CPT >= 8 || (CPT == 4 && NP <= 64) ? 2 : 4);
    static_assert(NTHR % PR == 0 && CPT >= 1 && NP % TR == 0, "Y splits evenly over the threads");
    __shared__ double xs[PR * S], ys[PR * S];
    __shared__ double sval[CSR_CHUNK];
    __shared__ int32_t scol[CSR_CHUNK];
    __shared__ int64_t rps[PR + 1];
    __shared__ double gmax[NTHR];

    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = p.n;
    const int64_t m = p.m;
    const int r = threadIdx.x / TR, tc = threadIdx.x % TR;
    // Panels, XCD by XCD: workgroups are dispatched round-robin over the chip's 8 XCDs
    // (workgroup b on XCD b % 8), each with its own L2.  Each XCD gets a contiguous range of
    // panels, and its workgroups take that range's panels in turn, so that the workgroups of
    // one L2 work on neighbouring panels at the same time and the rows of X that a stencil's
    // entries gather (the panel's neighbouring rows, shared by nearby panels) are fetched into
    // that L2 once rather than by every workgroup that needs them.
    const int64_t npanels = (m + PR - 1) / PR;
    const int G = gridDim.x;
    const int nx = G < 8 ? G : 8;
    const int xg = blockIdx.x % nx, slot = blockIdx.x / nx;
    const int nslot = (G - xg + nx - 1) / nx;  // workgroups on this workgroup's XCD
    const int64_t per = (npanels + nx - 1) / nx;
    const int64_t p0 = (int64_t)xg * per + slot;
    const int64_t p1 = ((int64_t)xg + 1) * per < npanels ? ((int64_t)xg + 1) * per : npanels;

    d4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
    int ti[TPW], tj[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int v = wv + u * WAVES < VT ? wv + u * WAVES : 0;
        const int t = v < T ? v : v - T;
        ti[u] = 16 * tile_row(NT, t);
        tj[u] = 16 * tile_col(NT, t);
    }
    bool bad = false;
    double bm = 0.0;

    for (int64_t pn = p0; pn < p1; pn += nslot) {
        const int64_t r0 = pn * PR;
        const int nr = (int)((m - r0 < PR) ? m - r0 : PR);
        __syncthreads();
        for (int idx = threadIdx.x; idx < PR * NP; idx += NTHR) {
            const int rr = idx / NP, cc = idx % NP;
            const int64_t row = r0 + rr;
            xs[rr * S + cc] = (row < m && cc < n) ? as_global(p.X)[row * p.ldx + cc] : 0.0;
        }
        if (threadIdx.x <= nr) rps[threadIdx.x] = as_global(p.brp)[r0 + threadIdx.x];
        __syncthreads();
        // entries of the panel: [lo, hi); row r's: [e0, e1) inside it
        const int64_t lo = rps[0], hi = rps[nr];
        const bool panel_ok = lo >= 0 && lo <= hi && hi <= p.bnnz;
        int64_t e0 = 0, e1 = 0;
        if (r < nr && panel_ok) {
            e0 = rps[r];
            e1 = rps[r + 1];
            if (!(e0 >= lo && e0 <= e1 && e1 <= hi)) {
                bad = true;
                e1 = e0;
            }
        }
        if (!panel_ok) bad = true;
        double y[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) y[q] = 0.0;
        double asum = 0.0;
        const int64_t hi_ok = panel_ok ? hi : lo;
        for (int64_t cs = lo; cs < hi_ok; cs += CSR_CHUNK) {
            const int cnt = (int)((hi_ok - cs < CSR_CHUNK) ? hi_ok - cs : CSR_CHUNK);
            __syncthreads();
            for (int i = threadIdx.x; i < cnt; i += NTHR) {
                const int32_t j = as_global(p.bcol)[cs + i];
                const bool jok = j >= 0 && (int64_t)j < m;
                if (!jok) bad = true;
                scol[i] = jok ? j : -1;
                sval[i] = as_global(p.bval)[cs + i];
            }
            __syncthreads();
            const int a = (int)((e0 > cs ? e0 : cs) - cs);
            const int b = (int)((e1 < cs + cnt ? e1 : cs + cnt) - cs);
            for (int e = a; e < b; e += GB) {
                double xv[GB][CPT], vv[GB];
                bool ok[GB];
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    const int j = (e + u < b) ? scol[e + u] : -1;
                    ok[u] = j >= 0;
                    vv[u] = ok[u] ? sval[e + u] : 0.0;
                    if constexpr (BG) {
                        const auto xr = as_global(p.X) + (int64_t)(ok[u] ? j : 0) * p.ldx;
#pragma unroll
                        for (int q = 0; q < CPT; ++q) {
                            const int cc = tc + TR * q;
                            xv[u][q] = (ok[u] && cc < n) ? xr[cc] : 0.0;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    if (ok[u]) {
                        if constexpr (BG) {
#pragma unroll
                            for (int q = 0; q < CPT; ++q) y[q] = __builtin_fma(vv[u], xv[u][q], y[q]);
                        }
                        if (EUC) asum += fabs(vv[u]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) ys[r * S + tc + TR * q] = y[q];
        if (EUC && tc == 0 && r < nr) bm = asum > bm ? asum : bm;
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < PR / 4; ++s4) {
            const int rr = 4 * s4 + (lane >> 4);
            const double *xrow = xs + rr * S + (lane & 15);
            const double *yrow = ys + rr * S + (lane & 15);
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int v = wv + u * WAVES;
                if (v < VT) {
                    const double bv = (BG && v < T) ? yrow[tj[u]] : xrow[tj[u]];
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xrow[ti[u]], bv, acc[u], 0, 0, 0);
                }
            }
        }
    }
    if (bad) *p.bad_b = 1;
    double *out = partials + (int64_t)blockIdx.x * SLOT + VOFF;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int v = wv + u * WAVES;
        if (v < VT) {
            // KIND 1: X^T B X at [0, E), X^T X at [E, 2 E)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) out[(int64_t)v * 256 + rr * 64 + lane] = acc[u][rr];
        }
    }
    if (EUC) {
        gmax[threadIdx.x] = bm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double g = 0.0;
            for (int i = 0; i < NTHR; ++i) g = gmax[i] > g ? gmax[i] : g;
            bmax[blockIdx.x] = g;
        }
    }
}

// Batched form (Euclidean): workgroup b takes the rows of task b; pass > 1 reads the Q.
template <int NP, int WAVES, bool F32>
__global__ void __launch_bounds__(WAVES * 64)
k_gram_lds_b(const BatchInst *__restrict__ insts, const BatchTask *__restrict__ tasks,
             double *__restrict__ partials, int pass, int final_gram)
{
    constexpr int NT = NP / 16;
    constexpr int64_t E = (int64_t)NT * (NT + 1) / 2 * 256;
    const BatchTask t = load_cview(tasks + blockIdx.x);
    const BatchInst I = load_cview(insts + t.inst);
    Problem p = I.p;
    if (pass >= 1) {  // the Gram of pass >= 1 reads the Q its substitution just wrote
        p.X = p.Q;
        p.ldx = p.ldq;
    }
    gram_lds_body<NP, WAVES, false, false, F32>(p, partials + (int64_t)blockIdx.x * E, nullptr, I.w.ctl, pass,
                                                final_gram, t.r0 / 16, (t.r1 + 15) / 16);
}

// ------------------------------------------------------------------------------------------
// Fixed-order reduction of the per-workgroup partial Grams in two launches: block (x, g) of the
// first adds partials p = 32g .. 32g+31 in increasing p for its 256 elements; the second adds
// those level-2 sums in increasing g and writes the reduced tiles.  (Two launches instead of an
// arrival counter: the kernel boundary orders the level-2 writes before their reads, where a
// counter would need a device-scope release per block.)
__global__ void __launch_bounds__(256)
k_reduce_l1(const double *__restrict__ partials, double *__restrict__ lvl2, int nparts, int64_t elems,
            const Ctl *__restrict__ ctl, int pass, int final_gram)
{
    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= elems) return;
    const int g = blockIdx.y;
    const int p0 = 32 * g, p1 = (p0 + 32 < nparts) ? p0 + 32 : nparts;
    double v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = (p0 + q < p1) ? partials[(int64_t)(p0 + q) * elems + e] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 32; ++q)
        if (p0 + q < p1) s += v[q];
    lvl2[(int64_t)g * elems + e] = s;
}

__global__ void __launch_bounds__(256)
k_reduce_l2(const double *__restrict__ lvl2, double *__restrict__ gsum, int nlvl2, int64_t elems,
            const Ctl *__restrict__ ctl, int pass, int final_gram)
{
    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= elems) return;
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= nlvl2; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = lvl2[(int64_t)(q + u) * elems + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < nlvl2; ++q) s += lvl2[(int64_t)q * elems + e];
    gsum[e] = s;
}

// Batched reduction: block (x, i) adds the partials of instance i's tasks t0 .. t1-1 in
// increasing order for its 256 elements (an instance has few tasks, so one level suffices).
__global__ void __launch_bounds__(256)
k_reduce_b(const BatchInst *__restrict__ insts, const double *__restrict__ partials, int64_t elems,
           int pass, int final_gram)
{
    const BatchInst I = load_cview(insts + blockIdx.y);
    const Ctl *ctl = I.w.ctl;
    if (!gate(ctl, pass)) return;
    if (!gram_needed(ctl, pass, final_gram)) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= elems) return;
    const int t1 = I.t1;
    double s = 0.0;
    int q = I.t0;
    for (; q + 8 <= t1; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partials[(int64_t)(q + u) * elems + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < t1; ++q) s += partials[(int64_t)q * elems + e];
    I.w.gsum[e] = s;
}

// ------------------------------------------------------------------------------------------
// Launchers
static int g_cu_count = 0;

static int cu_count()
{
    if (g_cu_count == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            g_cu_count = cus;
        else
            g_cu_count = 256;
    }
    return g_cu_count;
}

static bool uses_small(int np, bool oblique) { return np <= 64 && !oblique; }

int pass_grid(int64_t m, int np)
{
    const int cus = cu_count();
    if (np <= 32) {
        // workgroups of 4 waves on 64-row panels, persistent over the panels; two (n <= 32)
        // or four (n <= 16) fit a CU's LDS
        const int64_t panels = (m + 63) / 64;
        int64_t wg = (panels + 3) / 4;
        const int64_t cap = (np <= 16 ? 4 : 2) * (int64_t)cus;
        if (wg > cap) wg = cap;
        return (int)(wg < 1 ? 1 : wg);
    }
    if (np <= 64) {
        // one workgroup of 8 waves (32-row panels) per CU, persistent over the panels
        const int64_t panels = (m + 31) / 32;
        int64_t wg = (panels + 7) / 8;
        const int64_t cap = (int64_t)cus;
        if (wg > cap) wg = cap;
        return (int)(wg < 1 ? 1 : wg);
    }
    const int64_t panels = (m + 15) / 16;
    int64_t cap = (np <= 128 ? 2 : 1) * (int64_t)cus;
    int64_t wg = panels < cap ? panels : cap;
    return (int)(wg < 1 ? 1 : wg);
}

int64_t pass_partial_elems(int np, bool oblique_first)
{
    const int nt = np / 16;
    const int64_t e = (int64_t)upper_tiles(nt) * 256;
    return oblique_first ? 2 * e : e;
}

// Rows per panel of the fused kernel (64: 4 waves per workgroup, 32: 8 waves): 32 for the
// batched binary32 Gram (one panel is one binary32 chain) and the adjoint's transposed solve.
constexpr int kPanelRows = 32;
// Single problem: 64 for n <= 32, where one row per lane keeps all 64 lanes busy in the
// diagonal-block substitution; 32 for n <= 64, where a 64-row panel would not fit a wave's
// registers.  The binary32 Gram keeps its 32-row chains.
template <int NP>
constexpr int single_panel_rows() { return NP <= 32 ? 64 : 32; }

template <int NP, bool VEC>
static void launch_small_v(hipStream_t s, const Problem &p, const Work &w, int mode, int pass,
                           bool f32, int final_gram)
{
    constexpr int PR = single_panel_rows<NP>();
    dim3 grid(w.nwg), block(PR == 64 ? 256 : 512);
    if (mode == 0) {
        if (f32)
            hipLaunchKernelGGL((k_pass_tile<NP, 0, true, VEC, f32_chain_rows(NP), false>), grid,
                               dim3(f32_chain_rows(NP) == 64 ? 256 : 512), 0, s, p, p.Q, factor_of(w, NP, pass),
                               dinv_of(w, NP, pass), w.partials, w.ctl, pass, final_gram, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_pass_tile<NP, 0, false, VEC, PR, false>), grid, block, 0, s, p, p.Q, factor_of(w, NP, pass), dinv_of(w, NP, pass),
                               w.partials, w.ctl, pass, final_gram, nullptr, nullptr);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_pass_tile<NP, 1, false, VEC, PR, false>), grid, block, 0, s, p, p.Q, factor_of(w, NP, pass), dinv_of(w, NP, pass),
                           w.partials, w.ctl, pass, final_gram, nullptr, nullptr);
    } else if (mode == 5) {
        // minimum traffic: the whole factor history, passes 1 .. pass
        if constexpr (NP <= 32) {
            constexpr int nt = NP / 16;
            const size_t dyn = sizeof(double) * (size_t)(nt * (nt - 1) / 2) * 256 * (size_t)pass;
            hipLaunchKernelGGL((k_pass_tile<NP, 5, false, VEC, PR, false>), grid, block, dyn, s, p, p.Q,
                               factor_of(w, NP, 1), dinv_of(w, NP, 1), w.partials, w.ctl, pass, final_gram, nullptr,
                               nullptr);
        }
    } else {
        hipLaunchKernelGGL((k_pass_tile<NP, 2, false, VEC, PR, false>), grid, block, 0, s, p, p.Q, factor_of(w, NP, pass), dinv_of(w, NP, pass),
                           w.partials, w.ctl, pass, final_gram, nullptr, nullptr);
    }
}

template <int NP>
static hipError_t launch_small(hipStream_t s, const Problem &p, const Work &w, int mode, int pass,
                               bool f32, int final_gram)
{
    const bool aligned = (reinterpret_cast<uintptr_t>(p.X) & 15) == 0 && (p.ldx & 1) == 0 && p.ldx <= kBufMaxLd &&
                         (mode == 0 || ((reinterpret_cast<uintptr_t>(p.Q) & 15) == 0 && (p.ldq & 1) == 0 &&
                                        p.ldq <= kBufMaxLd));
    if (aligned && (p.n & 1) == 0)
        launch_small_v<NP, true>(s, p, w, mode, pass, f32, final_gram);
    else
        launch_small_v<NP, false>(s, p, w, mode, pass, f32, final_gram);
    return hipGetLastError();
}

template <int NP, int WAVES>
static hipError_t launch_gram_lds(hipStream_t s, const Problem &p, const Work &w, int pass,
                                  bool f32, bool obl, bool euc, int final_gram)
{
    dim3 grid(w.nwg), block(WAVES * 64);
    if (obl && euc)
        hipLaunchKernelGGL((k_gram_lds<NP, WAVES, true, true, false>), grid, block, 0, s, p,
                           w.partials, w.bmax, w.ctl, pass, final_gram);
    else if (obl)
        hipLaunchKernelGGL((k_gram_lds<NP, WAVES, true, false, false>), grid, block, 0, s, p,
                           w.partials, w.bmax, w.ctl, pass, final_gram);
    else if (f32)
        hipLaunchKernelGGL((k_gram_lds<NP, WAVES, false, false, true>), grid, block, 0, s, p,
                           w.partials, w.bmax, w.ctl, pass, final_gram);
    else
        hipLaunchKernelGGL((k_gram_lds<NP, WAVES, false, false, false>), grid, block, 0, s, p,
                           w.partials, w.bmax, w.ctl, pass, final_gram);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_wide(hipStream_t s, const Problem &p, const Work &w, int mode, int pass, int final_gram)
{
    const bool vec = (reinterpret_cast<uintptr_t>(p.X) & 15) == 0 && (p.ldx & 1) == 0 &&
                     (reinterpret_cast<uintptr_t>(p.Q) & 15) == 0 && (p.ldq & 1) == 0 && (p.n & 1) == 0 &&
                     p.ldx <= kBufMaxLd && p.ldq <= kBufMaxLd;
    dim3 grid(w.nwg), block(256);
    const double *Rt = factor_of(w, NP, pass), *dv = dinv_of(w, NP, pass);
    if (mode == 1 && vec)
        hipLaunchKernelGGL((k_pass_wide<NP, 1, true>), grid, block, 0, s, p, p.Q, Rt, dv, w.partials, w.ctl, pass, final_gram);
    else if (mode == 1)
        hipLaunchKernelGGL((k_pass_wide<NP, 1, false>), grid, block, 0, s, p, p.Q, Rt, dv, w.partials, w.ctl, pass, final_gram);
    else if (vec)
        hipLaunchKernelGGL((k_pass_wide<NP, 2, true>), grid, block, 0, s, p, p.Q, Rt, dv, w.partials, w.ctl, pass, final_gram);
    else
        hipLaunchKernelGGL((k_pass_wide<NP, 2, false>), grid, block, 0, s, p, p.Q, Rt, dv, w.partials, w.ctl, pass, final_gram);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_gram_wide(hipStream_t s, const Problem &p, const Work &w, int pass, bool f32,
                                   bool obl, bool euc, int final_gram)
{
    dim3 grid(w.nwg), block(gram_wide_threads(NP, obl, euc, f32));
    const BatchInst *ni = nullptr;
    const BatchTask *nt = nullptr;
    if constexpr (NP == 256) {
        if (f32)
            hipLaunchKernelGGL((k_gram_wide<NP, false, false, true, false>), grid, block, 0, s, p, w.partials,
                               w.bmax, w.ctl, pass, final_gram, ni, nt);
        else
            hipLaunchKernelGGL((k_gram_wide<NP, false, false, false, false>), grid, block, 0, s, p, w.partials,
                               w.bmax, w.ctl, pass, final_gram, ni, nt);
        return hipGetLastError();
    } else {
    if (obl && euc)
        hipLaunchKernelGGL((k_gram_wide<NP, true, true, false, false>), grid, block, 0, s, p, w.partials, w.bmax,
                           w.ctl, pass, final_gram, ni, nt);
    else if (obl)
        hipLaunchKernelGGL((k_gram_wide<NP, true, false, false, false>), grid, block, 0, s, p, w.partials, w.bmax,
                           w.ctl, pass, final_gram, ni, nt);
    else if (f32) {
        // the binary32 Gram of np <= 64 is formed by k_pass_tile
        if constexpr (NP == 128)
            hipLaunchKernelGGL((k_gram_wide<NP, false, false, true, false>), grid, block, 0, s, p, w.partials,
                               w.bmax, w.ctl, pass, final_gram, ni, nt);
        else
            return hipErrorInvalidValue;
    } else
        hipLaunchKernelGGL((k_gram_wide<NP, false, false, false, false>), grid, block, 0, s, p, w.partials, w.bmax,
                           w.ctl, pass, final_gram, ni, nt);
    return hipGetLastError();
    }
}

// n = 256 substitution Q = X R~^{-1} as a 2 x 2 block solve, still row-wise in blocked order:
// Q_1 = X_1 R~_11^{-1};  Q_2 = (X_2 - Q_1 R~_12) R~_22^{-1}  (columns 0..127 and 128..n-1).
static hipError_t launch_trsm_256(hipStream_t s, const Problem &p, const Work &w, int pass)
{
    const double *Rt = factor_of(w, 256, pass), *dv = dinv_of(w, 256, pass);
    hipLaunchKernelGGL(k_split256, dim3(16), dim3(256), 0, s, Rt, dv, w.Rsplit, w.ctl, pass);
    const double *R11 = w.Rsplit, *R22 = w.Rsplit + 128 * 128;
    const double *d11 = w.Rsplit + 2 * 128 * 128, *d22 = d11 + 128;
    const bool vec = (reinterpret_cast<uintptr_t>(p.X) & 15) == 0 && (p.ldx & 1) == 0 &&
                     (reinterpret_cast<uintptr_t>(p.Q) & 15) == 0 && (p.ldq & 1) == 0 && (p.n & 1) == 0 &&
                     p.ldx <= kBufMaxLd && p.ldq <= kBufMaxLd;
    const int cus = cu_count();
    Problem p1 = p;
    p1.n = 128;
    p1.np = 128;
    dim3 grid((unsigned)cus), block(256);
    const int n2 = p.n - 128;
    // Q_1 and X'_2 = X_2 - Q_1 R~_12 in one pass over the rows
    const WideProd pr{p.X + 128, p.ldx, p.Q + 128, p.ldq, Rt + 128, (int64_t)256, n2};
    if (vec)
        hipLaunchKernelGGL((k_pass_wide4<true>), grid, block, 0, s, p1, p1.Q, R11, d11, pr, w.ctl, pass);
    else
        hipLaunchKernelGGL((k_pass_wide4<false>), grid, block, 0, s, p1, p1.Q, R11, d11, pr, w.ctl, pass);
    Problem p3 = p;
    p3.n = n2;
    p3.np = 128;
    p3.X = p.Q + 128;
    p3.ldx = p.ldq;
    p3.Q = p.Q + 128;
    if (vec)
        hipLaunchKernelGGL((k_pass_wide<128, 2, true>), grid, block, 0, s, p3, p3.Q, R22, d22, w.partials, w.ctl, pass, 0);
    else
        hipLaunchKernelGGL((k_pass_wide<128, 2, false>), grid, block, 0, s, p3, p3.Q, R22, d22, w.partials, w.ctl, pass, 0);
    return hipGetLastError();
}

// Waves per workgroup of the CSR Gram: 4 up to n = 64 (five workgroups per CU: each one's
// staging barriers stall fewer waves; 27-point B at 10^6 x 64: 1.32 -> 1.15 ms per pass), 8 at
// n = 128; at n = 256 the 136 tiles take 16 waves (9 tiles, 72 accumulator registers each), and
// the first pass's two sets of tiles take two launches (KIND 2, then 3).
template <int NP>
static hipError_t launch_gram_csr(hipStream_t s, const Problem &p, const Work &w, int pass, bool euc, int final_gram)
{
    constexpr int W = NP <= 64 ? 4 : (NP == 256 ? 16 : 8);
    dim3 grid(w.nwg), block(W * 64);
    if (euc) {
        if constexpr (NP == 256) {
            hipLaunchKernelGGL((k_gram_csr<NP, W, 2>), grid, block, 0, s, p, w.partials, w.bmax, w.ctl, pass,
                               final_gram);
            hipLaunchKernelGGL((k_gram_csr<NP, W, 3>), grid, block, 0, s, p, w.partials, w.bmax, w.ctl, pass,
                               final_gram);
        } else {
            hipLaunchKernelGGL((k_gram_csr<NP, W, 1>), grid, block, 0, s, p, w.partials, w.bmax, w.ctl, pass,
                               final_gram);
        }
    } else {
        hipLaunchKernelGGL((k_gram_csr<NP, W, 0>), grid, block, 0, s, p, w.partials, w.bmax, w.ctl, pass, final_gram);
    }
    return hipGetLastError();
}

static hipError_t gram_generic(hipStream_t s, const Problem &p, const Work &w, int pass, bool f32,
                               bool obl, bool euc, int final_gram)
{
    if (obl && p.brp) {
        switch (p.np) {
        case 16: return launch_gram_csr<16>(s, p, w, pass, euc, final_gram);
        case 32: return launch_gram_csr<32>(s, p, w, pass, euc, final_gram);
        case 64: return launch_gram_csr<64>(s, p, w, pass, euc, final_gram);
        case 128: return launch_gram_csr<128>(s, p, w, pass, euc, final_gram);
        case 256: return launch_gram_csr<256>(s, p, w, pass, euc, final_gram);
        }
        return hipErrorInvalidValue;
    }
    switch (p.np) {
    case 16: return launch_gram_wide<16>(s, p, w, pass, f32, obl, euc, final_gram);
    case 32: return launch_gram_wide<32>(s, p, w, pass, f32, obl, euc, final_gram);
    case 64: return launch_gram_wide<64>(s, p, w, pass, f32, obl, euc, final_gram);
    case 128: return launch_gram_wide<128>(s, p, w, pass, f32, obl, euc, final_gram);
    case 256:
        if (!obl) return launch_gram_wide<256>(s, p, w, pass, f32, obl, euc, final_gram);
        return launch_gram_lds<256, 8>(s, p, w, pass, f32, obl, euc, final_gram);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pass(hipStream_t s, const Problem &p, const Work &w, int mode, int pass,
                       bool fp32_gram, bool oblique_gram, bool euclid_too)
{
    const int final_gram = (mode & 0x100) ? 1 : 0;
    mode &= 0xff;
    if (mode == 5 && (p.np > 32 || oblique_gram || pass < 1 || pass > SCQR_MAX_PASSES)) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (uses_small(p.np, oblique_gram)) {
        prof_before(s, mode == 0 ? (fp32_gram ? "gram_f32" : "gram") : mode == 1 ? "trsm_gram" : mode == 5 ? "trsm_gram_mt" : "trsm");
        switch (p.np) {
        case 16: e = launch_small<16>(s, p, w, mode, pass, fp32_gram, final_gram); break;
        case 32: e = launch_small<32>(s, p, w, mode, pass, fp32_gram, final_gram); break;
        case 64: e = launch_small<64>(s, p, w, mode, pass, fp32_gram, final_gram); break;
        default: e = hipErrorInvalidValue;
        }
        prof_after(s);
        return e;
    }
    if (p.np == 128 && mode == 1 && !oblique_gram) {
        prof_before(s, "trsm_gram");
        e = launch_wide<128>(s, p, w, 1, pass, final_gram);
        prof_after(s);
        return e;
    }
    // Generic path: separate substitution and Gram kernels.
    if (mode >= 1) {
        prof_before(s, "trsm");
        switch (p.np) {
        case 16: e = launch_small<16>(s, p, w, 2, pass, false, 0); break;
        case 32: e = launch_small<32>(s, p, w, 2, pass, false, 0); break;
        case 64: e = launch_small<64>(s, p, w, 2, pass, false, 0); break;
        case 128: e = launch_wide<128>(s, p, w, 2, pass, 0); break;
        case 256: e = launch_trsm_256(s, p, w, pass); break;
        default: e = hipErrorInvalidValue;
        }
        prof_after(s);
        if (e != hipSuccess) return e;
    }
    if (mode <= 1) {
        Problem pg = p;
        if (mode == 1) {  // the Gram reads the Q just written
            pg.X = p.Q;
            pg.ldx = p.ldq;
        }
        prof_before(s, oblique_gram ? (p.brp ? (euclid_too ? "gram_csr_first" : "gram_csr")
                                             : (euclid_too ? "gram_b_first" : "gram_b"))
                                    : (fp32_gram ? "gram_f32" : "gram"));
        e = gram_generic(s, pg, w, pass, fp32_gram, oblique_gram, euclid_too, final_gram);
        prof_after(s);
    }
    return e;
}

hipError_t launch_reduce(hipStream_t s, const Work &w, int pass, int64_t elems, int final_gram)
{
    dim3 grid((unsigned)((elems + 255) / 256), (unsigned)w.nlvl2), block(256);
    prof_before(s, "reduce");
    hipLaunchKernelGGL(k_reduce_l1, grid, block, 0, s, w.partials, w.lvl2, w.nwg, elems, w.ctl, pass, final_gram);
    hipLaunchKernelGGL(k_reduce_l2, dim3(grid.x), block, 0, s, w.lvl2, w.gsum, w.nlvl2, elems, w.ctl, pass,
                       final_gram);
    prof_after(s);
    return hipGetLastError();
}

// ---- batched launchers -------------------------------------------------------------------
template <int NP, bool VEC, int PR>
static void launch_small_b(hipStream_t s, const BatchClass &c, int mode, int pass, bool f32, int final_gram)
{
    dim3 grid((unsigned)c.ntasks), block(PR == 64 ? 256 : 512);
    if (mode == 0 && f32)  // the binary32 chain is one 32-row panel, whatever the tuning
        hipLaunchKernelGGL((k_pass_tile<NP, 0, true, VEC, kPanelRows, true>), grid, dim3(512), 0, s, Problem{}, nullptr,
                           nullptr, nullptr, c.partials, nullptr, pass, final_gram, c.insts, c.tasks);
    else if (mode == 0)
        hipLaunchKernelGGL((k_pass_tile<NP, 0, false, VEC, PR, true>), grid, block, 0, s, Problem{}, nullptr, nullptr, nullptr,
                           c.partials, nullptr, pass, final_gram, c.insts, c.tasks);
    else
        hipLaunchKernelGGL((k_pass_tile<NP, 1, false, VEC, PR, true>), grid, block, 0, s, Problem{}, nullptr, nullptr, nullptr,
                           c.partials, nullptr, pass, final_gram, c.insts, c.tasks);
}

template <int NP>
static void launch_small_bv(hipStream_t s, const BatchClass &c, int mode, int pass, bool f32, int final_gram)
{
    if (c.vec) {
        if (c.pr == 64)
            launch_small_b<NP, true, 64>(s, c, mode, pass, f32, final_gram);
        else
            launch_small_b<NP, true, 32>(s, c, mode, pass, f32, final_gram);
    } else {
        if (c.pr == 64)
            launch_small_b<NP, false, 64>(s, c, mode, pass, f32, final_gram);
        else
            launch_small_b<NP, false, 32>(s, c, mode, pass, f32, final_gram);
    }
}

template <int NP, int WAVES>
static void launch_big_b(hipStream_t s, const BatchClass &c, int mode, int pass, bool f32, int final_gram)
{
    dim3 grid((unsigned)c.ntasks);
    if (NP == 128 && mode == 1) {
        prof_before(s, "b_trsm_gram");
        if (c.vec)
            hipLaunchKernelGGL((k_pass_wide_b<128, 1, true>), grid, dim3(256), 0, s, c.insts, c.tasks, c.partials,
                               pass, final_gram);
        else
            hipLaunchKernelGGL((k_pass_wide_b<128, 1, false>), grid, dim3(256), 0, s, c.insts, c.tasks, c.partials,
                               pass, final_gram);
        prof_after(s);
        return;
    }
    if (mode >= 1) {
        prof_before(s, "b_trsm");
        hipLaunchKernelGGL((k_trsm_big_b<NP>), grid, dim3(256), 0, s, c.insts, c.tasks, pass);
        prof_after(s);
    }
    prof_before(s, f32 ? "b_gram_f32" : "b_gram");
    if constexpr (NP == 128) {
        if (f32)
            hipLaunchKernelGGL((k_gram_wide<NP, false, false, true, true>), grid,
                               dim3(gram_wide_threads(NP, false, false, true)), 0, s, Problem{},
                               c.partials, nullptr, nullptr, pass, final_gram, c.insts, c.tasks);
        else
            hipLaunchKernelGGL((k_gram_wide<NP, false, false, false, true>), grid,
                               dim3(gram_wide_threads(NP, false, false, false)), 0, s, Problem{},
                               c.partials, nullptr, nullptr, pass, final_gram, c.insts, c.tasks);
    } else if (f32) {
        hipLaunchKernelGGL((k_gram_lds_b<NP, WAVES, true>), grid, dim3(WAVES * 64), 0, s, c.insts, c.tasks,
                           c.partials, pass, final_gram);
    } else {
        hipLaunchKernelGGL((k_gram_lds_b<NP, WAVES, false>), grid, dim3(WAVES * 64), 0, s, c.insts, c.tasks,
                           c.partials, pass, final_gram);
    }
    prof_after(s);
}

hipError_t launch_pass_b(hipStream_t s, const BatchClass &c, int mode, int pass, bool fp32_gram, int final_gram)
{
    if (c.ntasks <= 0) return hipSuccess;
    if (c.np <= 64) {
        prof_before(s, mode == 0 ? (fp32_gram ? "b_gram_f32" : "b_gram") : "b_trsm_gram");
        switch (c.np) {
        case 16: launch_small_bv<16>(s, c, mode, pass, fp32_gram, final_gram); break;
        case 32: launch_small_bv<32>(s, c, mode, pass, fp32_gram, final_gram); break;
        case 64: launch_small_bv<64>(s, c, mode, pass, fp32_gram, final_gram); break;
        }
        prof_after(s);
        return hipGetLastError();
    }
    switch (c.np) {
    case 128: launch_big_b<128, 4>(s, c, mode, pass, fp32_gram, final_gram); break;
    case 256: launch_big_b<256, 8>(s, c, mode, pass, fp32_gram, final_gram); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_b(hipStream_t s, const BatchClass &c, int pass, int final_gram)
{
    if (c.ninst <= 0) return hipSuccess;
    const int64_t elems = pass_partial_elems(c.np, false);
    dim3 grid((unsigned)((elems + 255) / 256), (unsigned)c.ninst), block(256);
    prof_before(s, "b_reduce");
    hipLaunchKernelGGL(k_reduce_b, grid, block, 0, s, c.insts, c.partials, elems, pass, final_gram);
    prof_after(s);
    return hipGetLastError();
}

// ---- products and transposed solves used by the QR adjoint ---------------------------------
// Out = Base + SIGN * A B (TRANS: B read transposed), K the padded width of the factor.
template <int K, int NB, bool TRANS, int SIGN>
static void launch_mm_t(hipStream_t s, int64_t m, int ncols, int ka, const double *A, int64_t lda, const double *B,
                        int64_t ldb, const double *Base, int64_t ldbase, double *Out, int64_t ldo)
{
    const int cus = cu_count();
    int64_t panels = (m + 31) / 32;
    int64_t gx = panels < 2 * (int64_t)cus ? panels : 2 * (int64_t)cus;
    if (gx < 1) gx = 1;
    if constexpr (K >= 128) {
        dim3 grid((unsigned)gx, (unsigned)((ncols + 63) / 64)), block(256);
        hipLaunchKernelGGL((k_mm_breg<K, TRANS, SIGN>), grid, block, 0, s, m, ncols, ka, A, lda, B, ldb, Base, ldbase,
                           Out, ldo, (const Ctl *)nullptr, 0, 0);
    } else {
        dim3 grid((unsigned)gx, (unsigned)((ncols + NB - 1) / NB)), block(256);
        hipLaunchKernelGGL((k_mm<K, NB, TRANS, SIGN>), grid, block, 0, s, m, ncols, ka, A, lda, B, ldb, Base, ldbase,
                           Out, ldo, (const Ctl *)nullptr, 0, 0);
    }
}

hipError_t launch_mm(hipStream_t s, int np, int64_t m, int ncols, int ka, const double *A, int64_t lda,
                     const double *B, int64_t ldb, const double *Base, int64_t ldbase, double *Out, int64_t ldo)
{
    switch (np) {
    case 16: launch_mm_t<16, 16, false, 1>(s, m, ncols, ka, A, lda, B, ldb, Base, ldbase, Out, ldo); break;
    case 32: launch_mm_t<32, 32, false, 1>(s, m, ncols, ka, A, lda, B, ldb, Base, ldbase, Out, ldo); break;
    case 64: launch_mm_t<64, 64, false, 1>(s, m, ncols, ka, A, lda, B, ldb, Base, ldbase, Out, ldo); break;
    case 128: launch_mm_t<128, 64, false, 1>(s, m, ncols, ka, A, lda, B, ldb, Base, ldbase, Out, ldo); break;
    case 256: launch_mm_t<256, 32, false, 1>(s, m, ncols, ka, A, lda, B, ldb, Base, ldbase, Out, ldo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NP>
static void launch_solve_tile(hipStream_t s, const Problem &p, const double *Rp, const double *dinv, bool vec)
{
    const Ctl *nc = nullptr;
    const BatchInst *ni = nullptr;
    const BatchTask *nt = nullptr;
    double *np_ = nullptr;
    // 8 waves on 32-row panels, one workgroup per CU
    int64_t wg = ((p.m + 31) / 32 + 7) / 8;
    if (wg > cu_count()) wg = cu_count();
    dim3 grid((unsigned)(wg < 1 ? 1 : wg)), block(512);
    if (vec)
        hipLaunchKernelGGL((k_pass_tile<NP, 3, false, true, kPanelRows, false>), grid, block, 0, s, p, p.Q, Rp, dinv,
                           np_, nc, 0, 0, ni, nt);
    else
        hipLaunchKernelGGL((k_pass_tile<NP, 3, false, false, kPanelRows, false>), grid, block, 0, s, p, p.Q, Rp,
                           dinv, np_, nc, 0, 0, ni, nt);
}

static void launch_solve_wide(hipStream_t s, const Problem &p, const double *Rp, const double *dinv, bool vec)
{
    const Ctl *nc = nullptr;
    double *np_ = nullptr;
    dim3 grid((unsigned)cu_count()), block(256);
    if (vec)
        hipLaunchKernelGGL((k_pass_wide<128, 3, true>), grid, block, 0, s, p, p.Q, Rp, dinv, np_, nc, 0, 0);
    else
        hipLaunchKernelGGL((k_pass_wide<128, 3, false>), grid, block, 0, s, p, p.Q, Rp, dinv, np_, nc, 0, 0);
}

// Y <- X with X R~^T = Y, in place (row-major m x n, padded factor Rp of width np with identity
// padding, reciprocal diagonal dinv).  n = 256 is a 2 x 2 block solve:
// X_2 = Y_2 R~_22^{-T},  X_1 = (Y_1 - X_2 R~_12^T) R~_11^{-T}.
hipError_t launch_solve_t(hipStream_t s, int np, int64_t m, int n, double *Y, int64_t ldy, const double *Rp,
                          const double *dinv, double *Rsplit)
{
    Problem p{};
    p.m = m;
    p.n = n;
    p.np = np;
    p.X = Y;
    p.ldx = ldy;
    p.Q = Y;
    p.ldq = ldy;
    const bool vec = (reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (ldy & 1) == 0 && (n & 1) == 0 &&
                     ldy <= kBufMaxLd;
    switch (np) {
    case 16: launch_solve_tile<16>(s, p, Rp, dinv, vec); break;
    case 32: launch_solve_tile<32>(s, p, Rp, dinv, vec); break;
    case 64: launch_solve_tile<64>(s, p, Rp, dinv, vec); break;
    case 128: launch_solve_wide(s, p, Rp, dinv, vec); break;
    case 256: {
        hipLaunchKernelGGL(k_split256, dim3(16), dim3(256), 0, s, Rp, dinv, Rsplit, (const Ctl *)nullptr, 0);
        const double *R11 = Rsplit, *R22 = Rsplit + 128 * 128;
        const double *d11 = Rsplit + 2 * 128 * 128, *d22 = d11 + 128;
        const int n2 = n - 128;
        Problem p2 = p;
        p2.n = n2;
        p2.np = 128;
        p2.X = Y + 128;
        p2.Q = Y + 128;
        launch_solve_wide(s, p2, R22, d22, vec);
        launch_mm_t<128, 64, true, -1>(s, m, 128, n2, Y + 128, ldy, Rp + 128, 256, Y, ldy, Y, ldy);
        Problem p1 = p;
        p1.n = 128;
        p1.np = 128;
        launch_solve_wide(s, p1, R11, d11, vec);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// R = R~_q ... R~_1 for a factor of padded width np = 128 or 256: product q (2 <= q <= maxp) is
// P_q = R~_q P_{q-1} into Racc[q % 2] (P_1 = R~_1), launched for every q and skipped on the device
// beyond the applied passes.
hipError_t launch_rprod(hipStream_t s, const Work &w, int np, int maxp)
{
    for (int q = 2; q <= maxp; ++q) {
        const double *A = w.Rhist + (int64_t)(q - 1) * np * np;
        const double *B = q == 2 ? w.Rhist : w.Racc[(q - 1) & 1];
        if (np == 256)
            hipLaunchKernelGGL((k_mm_breg<256, false, 1>), dim3(8, 4), dim3(256), 0, s, (int64_t)256, 256, 256, A,
                               (int64_t)256, B, (int64_t)256, (const double *)nullptr, (int64_t)256, w.Racc[q & 1],
                               (int64_t)256, w.ctl, 0, q);
        else
            hipLaunchKernelGGL((k_mm_breg<128, false, 1>), dim3(4, 2), dim3(256), 0, s, (int64_t)128, 128, 128, A,
                               (int64_t)128, B, (int64_t)128, (const double *)nullptr, (int64_t)128, w.Racc[q & 1],
                               (int64_t)128, w.ctl, 0, q);
    }
    return hipGetLastError();
}

}  // namespace scqr
