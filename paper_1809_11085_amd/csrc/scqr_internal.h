// Internal declarations shared by the translation units of libscqr.so (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scqr.h"

namespace scqr {

constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Number of 16 x 16 tiles in the upper triangle of an NP x NP matrix (NP = 16 * NT).
__host__ __device__ constexpr int upper_tiles(int nt) { return nt * (nt + 1) / 2; }

// LDS row stride (in doubles) for panels read as Gram operands (lane l at row l / 16, column
// l % 16 of a 4 x 16 block): with S = 16 (mod 32) the two rows of each half-wave fall on disjoint
// halves of the 64 banks, and the bank-conflict counter of the Gram kernels reads 0 on gfx950
// (against about two conflict cycles per LDS instruction with S = np + 2).
__host__ __device__ constexpr int lds_stride_gram(int np) { return np % 64 == 16 ? np + 32 : np + 16; }

// Tile t (row-major enumeration of the upper triangle) -> block row I, block column J.
__host__ __device__ constexpr int tile_row(int nt, int t)
{
    int i = 0;
    while (t >= nt - i) {
        t -= nt - i;
        ++i;
    }
    return i;
}
__host__ __device__ constexpr int tile_col(int nt, int t)
{
    const int i = tile_row(nt, t);
    return t - (i * nt - i * (i - 1) / 2) + i;
}
__host__ __device__ inline void tile_ij(int nt, int t, int &I, int &J)
{
    I = tile_row(nt, t);
    J = tile_col(nt, t);
}

// Element e of a tile in the FP64 MFMA accumulator layout (lane l, register r; stored at
// e = r * 64 + l) -> row / column inside the 16 x 16 tile.  The 16x16x4 f64 instruction on
// gfx950 places D[i][j] in lane j + 16 * (i % 4), register i / 4.
__host__ __device__ inline void acc64_rc(int e, int &i, int &j)
{
    const int r = e >> 6, l = e & 63;
    i = (l >> 4) + 4 * r;
    j = l & 15;
}
// The 16x16x4 f32 instruction places D[i][j] in lane j + 16 * (i / 4), register i % 4.
__host__ __device__ inline void acc32_rc(int e, int &i, int &j)
{
    const int r = e >> 6, l = e & 63;
    i = 4 * (l >> 4) + r;
    j = l & 15;
}

// FP32-first option: rows accumulated in one binary32 MFMA chain of the first Gram before the
// chain's sum is added to the binary64 tiles, by padded width.  It is one panel of the kernel
// that forms that Gram (k_pass_tile: 32 rows for np <= 64; k_gram_wide: 64 rows at np = 128,
// 16 rows at np = 256; k_gram_lds flushes at the same counts), and the binary32 shift
// s32 = 11 ((k + 2) n u32 + n (n + 1) u) ||X||_2^2 takes this k.
__host__ __device__ constexpr int f32_chain_rows(int np) { return np <= 64 ? 32 : (np == 128 ? 64 : 16); }

// Padded width used by the kernels: the smallest of 16, 32, 64, 128, 256 that holds n.
inline int padded_n(int64_t n)
{
    int np = 16;
    while (np < n) np *= 2;
    return np;
}

// Device-side control block of one factorization (lives in the workspace).
struct Ctl {
    int32_t active;     // 0 once a breakdown / non-finite Gram stopped the schedule
    int32_t pass;       // number of passes whose R~ is ready
    int32_t last;       // pass whose TRSM is the final one (0 = not decided yet)
    int32_t redo_fp64;  // FP32-first: the first pass must be redone in binary64
    int32_t status;
    int32_t f32_pass;   // FP32-first: pass 1 factor came from the binary32 Gram
    int32_t bad_b;      // a Gram kernel met an out-of-range index of a CSR B
    int32_t vprev_pass; // pass whose power-iteration vector is in Work::vprev (0: none)
    double bnorm;       // ||B||_2 bound (1 for B = I)
};

// Per-problem description handed to the kernels.
struct Problem {
    int64_t m;
    int32_t n, np;
    const double *X;
    int64_t ldx;
    double *Q;
    int64_t ldq;
    double *R;
    int64_t ldr;
    const double *bdiag;   // tridiagonal B or nullptr
    const double *boff;
    const int64_t *brp;    // CSR B (row pointers, columns, values) or nullptr
    const int32_t *bcol;
    const double *bval;
    int64_t bnnz;
    int32_t *bad_b;        // CSR index errors are flagged here (the control block)
    int32_t zero;          // always 0; opaque to the compiler (keeps loads inside loops)
    double gram_depth;     // bound on the summation depth of this problem's Grams
};

// Workspace carve-out of one factorization.
struct Work {
    Ctl *ctl;
    double *G;          // np x np reduced Gram (both triangles)
    double *Ge;         // np x np Euclidean Gram of X for the oblique first-pass shift
    double *Rhist;      // SCQR_MAX_PASSES x np x np: factor R~ of each pass (identity padding)
    double *dhist;      // SCQR_MAX_PASSES x np: reciprocals of diag(R~) of each pass
    double *Racc[2];    // np x np ping-pong buffers for the final product R = R~_p ... R~_1
    double *partials;   // nwg x parts_elems
    double *lvl2;       // nlvl2 x parts_elems
    double *gsum;       // parts_elems: the reduced Gram tiles of the last reduction
    double *bmax;       // nwg per-workgroup Gershgorin maxima (oblique first pass)
    double *Rsplit;     // np = 256: R~_11, R~_22 (128 x 128 each) and their reciprocal diagonals
    double *vprev;      // np: the last power-iteration vector (start of the next pass's one)
    int nwg;            // workgroups (= partial count) of the pass kernels
    int nlvl2;          // level-2 partial count
    int64_t parts_elems;  // elements of one partial (tiles * 256, doubled for oblique pass 1)
};

// Factor and reciprocal diagonal used by the substitution of pass `pass` (slot 0 for pass 0).
__host__ __device__ inline const double *factor_of(const Work &w, int np, int pass)
{
    return w.Rhist + (int64_t)(pass > 1 ? pass - 1 : 0) * np * np;
}
__host__ __device__ inline const double *dinv_of(const Work &w, int np, int pass)
{
    return w.dhist + (int64_t)(pass > 1 ? pass - 1 : 0) * np;
}

// Schedule parameters copied to the Cholesky kernel by value.
struct SchedParams {
    int32_t schedule, shift_mode, precision, max_passes, final_gram, force_bd, zero_shift;
    int32_t oblique;
    double custom_alpha;
    double bnorm_user;
    double *trace;
    scqr_info *info;
};

// Read-only views in the constant address space.  The triangular factors, their reciprocal
// diagonals and the batched descriptors are never written while a kernel that reads them runs;
// loads through such a view of a wave-uniform address are scalar loads, also when the pointer
// came from memory (a batched descriptor) rather than from a restrict kernel argument.
template <class T>
using cview = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ cview<T> as_cview(const T *p)
{
    return (cview<T>)p;
}
// Global-address-space views of caller matrices: pointers taken from a descriptor in memory
// would otherwise be accessed with flat instructions.
template <class T>
using gview = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gview<T> as_global(T *p)
{
    return (gview<T>)p;
}
// Raw buffer views of a row range of a row-major matrix: a 128-bit buffer access whose byte
// offset (from the resource base) is at or beyond num_records reads zeros and writes nothing, so
// rows past the end and padding columns need no per-lane clamping (offsets are given in 32 bits;
// callers keep a panel within 2^31 bytes, see kBufMaxLd).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kBufOut = 0x80000000u;    // an offset beyond any resource built here
constexpr int64_t kBufMaxLd = (int64_t)1 << 21;  // leading dimensions (doubles) the buffer path takes
// Resource over the rows [r0, m) of an n-column matrix with leading dimension ld (doubles).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const double *base, int64_t ld, int64_t r0,
                                                            int64_t m, int n)
{
    const int64_t rem = ((m - r0 - 1) * ld + n) * 8;
    const int32_t nrec = rem > 0x7fffffff ? 0x7fffffff : (int32_t)rem;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base + r0 * ld), (short)0, nrec, 0x00020000);
}
// Workgroup barrier that orders LDS accesses only.  Global loads and stores in flight stay in
// flight across it; __syncthreads() also orders global memory and therefore waits for every
// outstanding global access (on gfx950 loads and stores share one counter).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// AUX: cache policy of the access (0: default; kBufStream: non-temporal, for data that a
// kernel streams once and that is not read again before the kernel ends).
constexpr int kBufStream = 2;
template <int AUX = 0>
__device__ __forceinline__ double2 buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, uint32_t off, double2 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, AUX);
}

// A trivially copyable descriptor loaded as 8-byte words through a constant view.
template <class T>
__device__ __forceinline__ T load_cview(const T *p)
{
    static_assert(sizeof(T) % 8 == 0, "descriptor size must be a multiple of 8 bytes");
    constexpr int W = (int)(sizeof(T) / 8);
    const cview<unsigned long long> src = as_cview(reinterpret_cast<const unsigned long long *>(p));
    unsigned long long w[W];
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = src[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// ---- batched factorization: instances grouped into classes of equal padded width np ----
// One instance (entry of a device-resident array).  p.X / p.Q / p.R / p.m / p.n are the
// instance's; w holds its control block, factors, reciprocal diagonals and reduced Gram.
struct BatchInst {
    Problem p;
    Work w;
    scqr_info *info;
    int32_t t0, t1;     // its tasks, which are also its partial-Gram slots, in the class
    int32_t pad[2];
};
// Rows [r0, r1) of one instance, processed by one workgroup of a pass kernel; r0 is a
// multiple of kBatchRowAlign.
struct BatchTask {
    int32_t inst;
    int32_t pad;
    int64_t r0, r1;
};
constexpr int kBatchRowAlign = 64;
struct BatchClass {
    int np;
    int ninst, ntasks;
    const BatchInst *insts;   // device
    const BatchTask *tasks;   // device
    double *partials;         // ntasks x pass_partial_elems(np, false)
    bool vec;                 // every instance allows 16-byte accesses of X and Q
    int pr;                   // np <= 64: rows per wave panel of the fused pass (32 or 64)
};
hipError_t launch_init_b(hipStream_t s, const BatchClass &c);
hipError_t launch_pass_b(hipStream_t s, const BatchClass &c, int mode, int pass, bool fp32_gram,
                         int final_gram);
hipError_t launch_reduce_b(hipStream_t s, const BatchClass &c, int pass, int final_gram);
hipError_t launch_chol_b(hipStream_t s, const BatchClass &c, const SchedParams &sp, int pass,
                         int variant);
hipError_t launch_finalize_b(hipStream_t s, const BatchClass &c);

// ---- launchers (each enqueues on `stream`, returns hipSuccess or the launch error) ----
int pass_grid(int64_t m, int np);
int64_t pass_partial_elems(int np, bool oblique_first);

// mode 0: Gram of X only; 1: Q = X R~^{-1} and Gram of Q; 2: Q = X R~^{-1} only; 5 (n <= 32,
// B = I): minimum traffic, Q of this pass recomputed from X through the factors of passes
// 1 .. pass, written only by the last pass, and its Gram.  Bit 0x100
// of mode asks for the Gram of the final pass too (final_gram option).
// `pass` selects the predicate on the control block (0 = unconditional, -1 = FP64 redo).
hipError_t launch_pass(hipStream_t s, const Problem &p, const Work &w, int mode, int pass,
                       bool fp32_gram, bool oblique_gram, bool euclid_too);
hipError_t launch_reduce(hipStream_t s, const Work &w, int pass, int64_t elems, int final_gram);
hipError_t launch_chol(hipStream_t s, const Problem &p, const Work &w, const SchedParams &sp,
                       int pass, int variant);
hipError_t launch_init(hipStream_t s, const Problem &p, const Work &w, const SchedParams &sp);
hipError_t launch_gram_out(hipStream_t s, const Work &w, int np, int n, double *G, int64_t ldg);
hipError_t launch_set_factor(hipStream_t s, const Work &w, int np, int n, const double *R,
                             int64_t ldr);
hipError_t launch_final_omega(hipStream_t s, const Problem &p, const Work &w,
                              const SchedParams &sp);
// maxp: the most passes the schedule can apply (the n = 256 product is one launch per pass).
hipError_t launch_finalize_r(hipStream_t s, const Problem &p, const Work &w, int maxp);
hipError_t launch_rprod(hipStream_t s, const Work &w, int np, int maxp);

// QR adjoint
// Out = Base + A B for the padded width np (Base may be null or equal Out; A must not overlap Out).
hipError_t launch_mm(hipStream_t s, int np, int64_t m, int ncols, int ka, const double *A, int64_t lda,
                     const double *B, int64_t ldb, const double *Base, int64_t ldbase, double *Out, int64_t ldo);
// Y <- X with X R~^T = Y in place; Rp is the np x np factor with identity padding, Rsplit scratch
// of 2 * 128 * 128 + 256 doubles for np = 256.
hipError_t launch_solve_t(hipStream_t s, int np, int64_t m, int n, double *Y, int64_t ldy, const double *Rp,
                          const double *dinv, double *Rsplit);
hipError_t launch_backward(hipStream_t s, int64_t m, int n, const double *Q, int64_t ldq,
                           const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                           const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws);
size_t backward_ws_bytes(int64_t m, int n);

// profiling hooks (api.hip)
void prof_before(hipStream_t s, const char *name);
void prof_after(hipStream_t s);

}  // namespace scqr
