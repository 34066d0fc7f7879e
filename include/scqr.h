/*
 * scqr.h — shifted Cholesky QR on AMD MI355X (gfx950): the C ABI of libscqr.so.
 *
 * Computes the thin QR factorization X = Q R of a tall-skinny X (m x n, m >= n, n <= 256),
 * optionally in the oblique inner product (x, y)_B = x^T B y of an SPD B, following
 * Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, "Shifted CholeskyQR for computing the QR
 * factorization of ill-conditioned matrices":
 *   - Algorithm 1 (shiftedCholeskyQR): A = X^T X, R = chol(A + sI), Q = X R^{-1};
 *   - Algorithm 3 (shiftedCholeskyQR3): one shifted pass, then CholeskyQR2;
 *   - Algorithm 2 (iterated CholeskyQR, shift only on breakdown);
 *   - Algorithm 5 (shiftedCholeskyQR3 in the B inner product, B tridiagonal here).
 * The shift is s = 11 (m n + n (n+1)) u ||X||_2^2 (equation (eq:finds2)) or, for B != I,
 * s = 11 (2 m sqrt(m n) + n (n+1)) u ||X||_2^2 ||B||_2 (equation (eq:finds2B)), u = 2^-53.
 *
 * Conventions shared by every entry point:
 *   - All matrix pointers are DEVICE pointers (HBM), row-major, with explicit leading
 *     dimensions (ld >= number of columns).  The caller owns and allocates every buffer
 *     (inputs, outputs, workspace, info); the library never allocates device memory on these
 *     paths and keeps no state between calls.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All work is
 *     enqueued on it; nothing synchronizes with the host.
 *   - Argument errors (shapes, null pointers, leading dimensions, workspace too small, n above
 *     the supported maximum) are returned synchronously and enqueue nothing.
 *   - Numerical outcomes (Cholesky breakdown, non-convergence, non-finite values) are written
 *     asynchronously into the caller's device-side scqr_info record; read it after the
 *     stream has completed.
 *   - Calls are re-entrant: concurrent calls must use distinct workspaces and outputs.
 */
#ifndef SCQR_H
#define SCQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCQR_MAX_N 256
#define SCQR_MAX_PASSES 16

typedef enum {
    SCQR_OK = 0,
    SCQR_E_INVALID = 1,       /* bad argument (shape, pointer, leading dimension, option)     */
    SCQR_E_WORKSPACE = 2,     /* workspace smaller than scqr_*_workspace_bytes() reported     */
    SCQR_E_UNSUPPORTED = 3,   /* valid request outside what the library implements            */
    SCQR_E_HIP = 4,           /* a HIP runtime call failed                                    */
    SCQR_E_BREAKDOWN = 5,     /* a Cholesky factorization broke down (Algorithm 2 test)       */
    SCQR_E_NOT_CONVERGED = 6, /* adaptive schedule hit max_passes without its stopping test   */
    SCQR_E_NONFINITE = 7      /* a Gram matrix contained NaN or Inf                           */
} scqr_status;

/* Pass schedule. */
enum {
    SCQR_SCHED_FIXED3 = 0,   /* Algorithm 3 / 5: shifted pass, then two unshifted passes     */
    SCQR_SCHED_ADAPTIVE = 1, /* Algorithm 3 followed by Algorithm 2 continuation: later passes
                                shift only when their Cholesky breaks down; a pass is the last
                                one when it ran unshifted on a Gram with ||A - I||_F <= 1/2   */
    SCQR_SCHED_CHOLQR2 = 2,  /* two unshifted passes (CholeskyQR2)                           */
    SCQR_SCHED_ITERATED = 3  /* Algorithm 2 from the first pass (shift only on breakdown)     */
};

/* Shift of a shifted pass. */
enum {
    SCQR_SHIFT_PAPER = 0,  /* (eq:finds2)/(eq:finds2B) with ||.||_2^2 from a power iteration  */
    SCQR_SHIFT_FRO = 1,    /* the same with ||X||_F^2 in place of ||X||_2^2 (Section 4.1)    */
    SCQR_SHIFT_SMALL = 2,  /* s = u ||X||_2^2 (||B||_2): remark after Table 3; no guarantee   */
    SCQR_SHIFT_CUSTOM = 3, /* s = custom_alpha ||X||_2^2 (||B||_2)                            */
    SCQR_SHIFT_DEPTH = 4   /* s = 11 (d n + n (n+1)) u ||X||_2^2: (eq:finds2) with the gamma_m
                              bound of the Gram (Section 3.1.1) replaced by gamma_d, d a bound
                              on the summation depth of the library's Gram for this launch
                              (rows one workgroup accumulates plus the fixed-order reductions;
                              reported in scqr_info.gram_depth).  Not in the paper, which leaves
                              a smaller safe shift open (remark after Table 3, Section 8).
                              Euclidean inner product only. */
};

/* Arithmetic of the first (preconditioning) pass. */
enum {
    SCQR_PREC_FP64 = 0,
    SCQR_PREC_FP32_FIRST = 1 /* first Gram in binary32 MFMA (binary64 reduction) with shift
                                s32 = 11 ((k+2) n u32 + n (n+1) u) ||X||_2^2, k the rows of one
                                binary32 chain (32 for n <= 64, 64 for n <= 128, 16 beyond),
                                u32 = 2^-24; if s32 > ||X||_2^2 / 100 or its
                                Cholesky breaks down, that pass is redone in binary64.  Not in
                                the paper; Euclidean inner product only. */
};

typedef struct {
    int32_t schedule;       /* SCQR_SCHED_*, default ADAPTIVE                                 */
    int32_t shift_mode;     /* SCQR_SHIFT_*, default PAPER                                    */
    int32_t precision;      /* SCQR_PREC_*, default FP64                                      */
    int32_t max_passes;     /* 1..SCQR_MAX_PASSES cap for ADAPTIVE/ITERATED, default 6        */
    int32_t final_gram;     /* 1: also form the Gram of the final Q and report omega_fro      */
    int32_t debug_force_breakdown_pass; /* >0: the Cholesky of that pass reports breakdown    */
    int32_t debug_zero_shift;           /* 1: every shift is zero                             */
    int32_t recompute;      /* 1: minimum-traffic passes (n <= 32, B = I; not in the paper).  A
                               pass before the last recomputes its input Q from X through the
                               factors of the earlier passes instead of reading a stored Q, and
                               writes no Q; only the last pass writes Q.  HBM traffic
                               8 (p + 2) m n bytes for p passes instead of 8 (2 p + 1) m n, at
                               p (p - 1) / 2 extra substitutions; Q, R and info equal those of
                               the default (0: each pass stores Q) bit for bit.  X is read by
                               every pass, so it must not change until the call completes (Q
                               may still alias X).  After a breakdown or a non-finite Gram
                               Q is not written (the default leaves the last completed pass's
                               Q).  Other shapes and the batched call: SCQR_E_UNSUPPORTED. */
    double custom_alpha;    /* SCQR_SHIFT_CUSTOM: s = custom_alpha ||X||_2^2 (||B||_2)        */
    double bnorm;           /* > 0: caller's bound on ||B||_2; else the Gershgorin bound      */
    double *trace;          /* nullable device buffer of max_passes * 2 * n * n doubles: for
                               pass p (0-based) the input Gram at trace[(2p) n n] and the
                               triangular factor R~ of that pass at trace[(2p+1) n n]          */
} scqr_opts;

/* Result record, written on the stream into caller-owned DEVICE memory. */
typedef struct {
    int32_t status;         /* scqr_status                                                    */
    int32_t passes;         /* Cholesky QR passes whose R~ was applied                        */
    int32_t shifted_mask;   /* bit p-1 set: pass p used a shift                               */
    int32_t breakdown_mask; /* bit p-1 set: a Cholesky of pass p broke down                   */
    int32_t fell_back_fp64; /* FP32_FIRST: the binary32 first pass was redone in binary64     */
    int32_t reserved;
    double shift[SCQR_MAX_PASSES];    /* shift used by pass p (0 if unshifted)                */
    double norm2sq[SCQR_MAX_PASSES];  /* ||.||_2^2 estimate behind that shift (0 if none)    */
    double gram_dev[SCQR_MAX_PASSES]; /* ||A_p - I||_F of the input Gram of pass p            */
    double omega_fro;       /* final_gram: ||Q^T Q - I||_F (or Q^T B Q) from the device Gram  */
    double bnorm;           /* ||B||_2 bound used (1 for B = I)                               */
    double gram_depth;      /* bound on the summation depth of the binary64 Grams (the d of
                               SCQR_SHIFT_DEPTH; reported for every shift mode)                */
} scqr_info;

/* Optional SPD operator B of the oblique inner product (Section 5).  NULL or kind NONE means
 * B = I.  The caller guarantees that B is symmetric positive definite.
 *   TRIDIAG: B symmetric tridiagonal with diag[m] and off[m-1] (device pointers).
 *   CSR: general sparse B in compressed sparse row form, the storage of the sparse B of
 *        Section 7 (device pointers): the entries of row i are col[e], val[e] for
 *        e = row_ptr[i] .. row_ptr[i+1]-1, row_ptr has m + 1 entries with row_ptr[0] = 0 and
 *        row_ptr[m] = nnz, both triangles are stored, the order inside a row is free.  (B x)_i
 *        is summed in storage order.  The indices live on the device and are checked by the
 *        kernels that read them: an entry whose row pointers leave [0, nnz] or decrease, or
 *        whose column leaves [0, m), is skipped, and scqr_qr reports SCQR_E_INVALID in info
 *        (scqr_gram has no status record: the Gram then lacks those entries).  The shift's
 *        ||B||_2 bound is the largest absolute row sum (Gershgorin) unless opts.bnorm > 0. */
enum { SCQR_B_NONE = 0, SCQR_B_TRIDIAG = 1, SCQR_B_CSR = 2 };
typedef struct {
    int32_t kind;
    int32_t reserved;
    const double *diag;      /* TRIDIAG */
    const double *off;       /* TRIDIAG */
    const int64_t *row_ptr;  /* CSR */
    const int32_t *col;      /* CSR */
    const double *val;       /* CSR */
    int64_t nnz;             /* CSR: number of stored entries (row_ptr[m]) */
} scqr_spd_op;

/* Fills *opts with the defaults listed above. */
void scqr_default_opts(scqr_opts *opts);

/* Human-readable name of a status code (static storage). */
const char *scqr_status_string(scqr_status s);

/* Workspace size in bytes for scqr_qr / scqr_gram / scqr_trsm at this shape (B may be NULL,
 * opts may be NULL for defaults).  Returns SCQR_E_INVALID for unsupported shapes. */
scqr_status scqr_workspace_bytes(int64_t m, int64_t n, const scqr_spd_op *B,
                                 const scqr_opts *opts, size_t *bytes);

/*
 * Thin QR factorization X = Q R by shifted Cholesky QR (Algorithms 1-3, 5).
 *   X   m x n, ldx >= n, read only (unless Q aliases it).
 *   Q   m x n, ldq >= n, output; may alias X exactly (Q == X and ldq == ldx) for in-place use.
 *   R   n x n, ldr >= n, output, upper triangular with positive diagonal; the strictly lower
 *       triangle is written with zeros.  Must not alias X, Q or the workspace.
 *   ws  workspace of at least scqr_workspace_bytes() bytes, 256-byte aligned.
 *   info device pointer to one scqr_info, written on the stream.
 * With B of kind TRIDIAG or CSR, Q^T B Q = I instead of Q^T Q = I (Algorithm 5; passes 2 and
 * later use the B-Gram Q^T B Q).
 */
scqr_status scqr_qr(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                    const scqr_spd_op *B, double *Q, int64_t ldq, double *R, int64_t ldr,
                    void *ws, size_t ws_bytes, const scqr_opts *opts, scqr_info *info);

/*
 * scqr_qr without a workspace argument and without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and status codes are those of scqr_qr; the
 * workspace is a static device array of SCQR_NOALLOC_SCRATCH_BYTES bytes inside the library
 * (one per GPU, held until the process ends; its device address is looked up once per device
 * on the first call there, with that device current).  Shapes whose workspace
 * (scqr_workspace_bytes) exceeds it return SCQR_E_WORKSPACE before anything is enqueued: at
 * most n <= 64 for any m, Euclidean or tridiagonal B, on a GPU of up to 256 compute units.  The
 * call allocates nothing (no hipMalloc, no library allocation) and enqueues the same kernels
 * as scqr_qr, with the same results bit for bit.  Every call on one GPU uses the same scratch:
 * calls that overlap in time on one GPU (other streams, other host threads) race and must be
 * serialized by the caller.  Nothing in the scratch needs to start at zero (the first kernel
 * of a call initialises the control state).
 */
#define SCQR_NOALLOC_SCRATCH_BYTES (16u << 20)
scqr_status scqr_qr_noalloc(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                            const scqr_spd_op *B, double *Q, int64_t ldq, double *R, int64_t ldr,
                            const scqr_opts *opts, scqr_info *info);

/*
 * Gram matrix G = X^T X (equation (eq:gram)), or X^T B X for tridiagonal or CSR B (Algorithm 4
 * line 1): the split-m SYRK of one pass with a fixed-order reduction across workgroups.  G is
 * n x n, ldg >= n, both triangles written (the upper triangle mirrored).
 */
scqr_status scqr_gram(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                      const scqr_spd_op *B, double *G, int64_t ldg, void *ws, size_t ws_bytes);

/*
 * Triangular solve Q = X R^{-1} row by row (Algorithm 1 line 4): each row q_i^T R = x_i^T is
 * solved by forward substitution (multiplication by the reciprocal of the diagonal).  R upper
 * triangular n x n with nonzero diagonal (only the upper triangle is read).  Q may alias X.
 */
scqr_status scqr_trsm(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                      const double *R, int64_t ldr, double *Q, int64_t ldq, void *ws,
                      size_t ws_bytes);

/*
 * Tuning of the batched schedule (not in the paper).  Instances are grouped into classes by
 * padded width (index c = 0..4 for 16, 32, 64, 128, 256); the rows of a class are cut into tasks,
 * one workgroup each.  A zero field takes the library default.
 *   rows_per_task[c]  rows of one task, rounded up to a multiple of 64; default: about 4096
 *                     tasks per class, at least 1024 rows per task.
 *   panel_rows[c]     classes of width <= 64 only: rows per wave panel of the fused pass, 32
 *                     (8 waves per workgroup) or 64 (4 waves); default 32.
 * The results do not depend on the tuning except through the rounding of the Gram sums (the
 * row partition changes the summation order).
 */
typedef struct {
    int64_t rows_per_task[5];
    int32_t panel_rows[5];
    int32_t reserved[3];
} scqr_batched_tuning;

/*
 * Batched QR of independent problems X_i (m_i x n_i, row-major).  m, n and the leading
 * dimensions ldx, ldq, ldr are host arrays of `batch` entries (ldx, ldq or ldr NULL: ld = n_i;
 * otherwise ld_i >= n_i); X, Q, R are host arrays of device pointers.  Every instance runs the
 * schedule in opts and writes its own infos[i] (device array of batch records).  Q_i may alias
 * X_i exactly (same pointer and leading dimension).  Workspace from
 * scqr_batched_workspace_bytes() with the same shapes, options and tuning (tune may be NULL).
 * The call copies the instance and task descriptors to the head of the workspace (an enqueued
 * host-to-device copy from library-owned pinned memory) and then enqueues the schedule; for
 * repeated calls on the same buffers, or under graph capture, use the batched plan below.
 */
scqr_status scqr_batched_workspace_bytes(int32_t batch, const int64_t *m, const int64_t *n,
                                         const scqr_opts *opts, const scqr_batched_tuning *tune,
                                         size_t *bytes);
scqr_status scqr_qr_batched(void *stream, int32_t batch, const int64_t *m, const int64_t *n,
                            const double *const *X, const int64_t *ldx, double *const *Q,
                            const int64_t *ldq, double *const *R, const int64_t *ldr, void *ws,
                            size_t ws_bytes, const scqr_opts *opts,
                            const scqr_batched_tuning *tune, scqr_info *infos);

/*
 * Batched plan: the batched factorization of one fixed set of buffers, for repeated calls and
 * for capture in a HIP graph.
 *   scqr_batched_plan_create  validates and plans on the host (arguments as scqr_qr_batched,
 *                             buffers included) and keeps the descriptor image in pinned host
 *                             memory that the plan allocates; no device work.
 *   scqr_batched_plan_upload  enqueues the copy of the descriptors to the head of ws on stream
 *                             (once, and again only if the workspace was overwritten).
 *   scqr_batched_plan_run     enqueues the schedule on stream: kernel launches only (no copy,
 *                             memset, allocation or host wait), so it may be captured in a graph
 *                             and replayed; each run re-initialises every instance's state.
 *   scqr_batched_plan_tuning  the tuning in effect (rows per task and panel rows per class) and
 *                             the number of tasks per class (ntasks may be NULL).
 *   scqr_batched_plan_destroy waits for the plan's upload, frees its host memory (not ws).
 * Runs of one plan, or of plans sharing a workspace, must not overlap in time.
 */
typedef struct scqr_batched_plan_s *scqr_batched_plan;
scqr_status scqr_batched_plan_create(int32_t batch, const int64_t *m, const int64_t *n,
                                     const double *const *X, const int64_t *ldx, double *const *Q,
                                     const int64_t *ldq, double *const *R, const int64_t *ldr,
                                     void *ws, size_t ws_bytes, const scqr_opts *opts,
                                     const scqr_batched_tuning *tune, scqr_info *infos,
                                     scqr_batched_plan *plan);
scqr_status scqr_batched_plan_upload(scqr_batched_plan plan, void *stream);
scqr_status scqr_batched_plan_run(scqr_batched_plan plan, void *stream);
scqr_status scqr_batched_plan_tuning(scqr_batched_plan plan, scqr_batched_tuning *tune,
                                     int32_t *ntasks);
scqr_status scqr_batched_plan_destroy(scqr_batched_plan plan);

/*
 * QR adjoint (reverse-mode derivative of X -> (Q, R) for the thin QR with positive diagonal):
 *   M = R dR^T - dQ^T Q,  dX = (dQ + Q copyltu(M)) R^{-T},
 * copyltu(M)_ij = M_{max(i,j), min(i,j)}.  dQ (m x n) and dR (n x n, only its upper triangle
 * is read) may be NULL (zero).  dX m x n output; may alias dQ.  Row-major, explicit lds.
 */
scqr_status scqr_backward_workspace_bytes(int64_t m, int64_t n, size_t *bytes);
scqr_status scqr_qr_backward(void *stream, int64_t m, int64_t n, const double *Q, int64_t ldq,
                             const double *R, int64_t ldr, const double *dQ, int64_t lddq,
                             const double *dR, int64_t lddr, double *dX, int64_t lddx, void *ws,
                             size_t ws_bytes);

/*
 * Kernel timing for measurement.  While enabled, every kernel the library enqueues is
 * bracketed by HIP events recorded on the launch stream (events are created on first use, so
 * keep this off on latency-critical paths).  scqr_profile_read() synchronizes on the
 * recorded events and returns one record per launch, in enqueue order (name and duration in
 * milliseconds; a launch that its device-side predicate skipped shows a near-zero duration),
 * then clears the record.  *count receives the number of records available, which may exceed
 * capacity (only the first `capacity` are copied).
 */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} scqr_kernel_stat;
scqr_status scqr_profile_enable(int32_t on);
scqr_status scqr_profile_read(scqr_kernel_stat *stats, int32_t capacity, int32_t *count);

/*
 * Device ceilings for the roofline figures (no part of a factorization).  All pointers are
 * device pointers, 16-byte aligned; nbytes a positive multiple of 16; grid = workgroups of 256
 * threads (0 selects 2048).  Time them with events on `stream`.
 *   scqr_peak_copy   dst[i] = src[i] over nbytes; variant bits 0-1 select 1, 2, 4 or 8
 *                    16-byte chunks per thread and step, bit 2 non-temporal stores.
 *   scqr_peak_read   reads nbytes; sink receives grid * 256 doubles (per-thread sums).
 *   scqr_peak_write  writes nbytes (variant as for the copy).
 *   scqr_peak_fp64   kind 0: FP64 MFMA 16x16x4 (2048 flops per instruction), kind 1: FP64
 *                    FMA (2 flops per lane): grid workgroups of four waves, each running
 *                    `iters` rounds of 8 independent instructions; sink as for the read.
 * Return SCQR_E_INVALID for bad arguments (nothing enqueued), SCQR_E_HIP on a launch error.
 */
scqr_status scqr_peak_copy(void *stream, const void *src, void *dst, int64_t nbytes, int32_t variant,
                           int32_t grid);
scqr_status scqr_peak_read(void *stream, const void *src, int64_t nbytes, int32_t variant, int32_t grid,
                           double *sink);
scqr_status scqr_peak_write(void *stream, void *dst, int64_t nbytes, int32_t variant, int32_t grid);
scqr_status scqr_peak_fp64(void *stream, int32_t kind, int32_t iters, int32_t grid, double *sink);

/* Build identification: a static string naming the target architecture and version. */
const char *scqr_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* SCQR_H */
