/*
 * CPU oracle for shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
 * "Shifted CholeskyQR for computing the QR factorization of ill-conditioned matrices").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library.  The GPU library never links, calls or includes it, and it
 * shares no code, header, table or helper with the GPU library.
 *
 * Plain, slow, obviously correct IEEE binary64 loops, compiled without floating-point
 * contraction (-ffp-contract=off), so every + and * rounds once as in the paper's error model
 * (Section 3, u = 2^-53).  OpenMP only distributes independent outputs (Gram entries, rows
 * of Q); the summation order of every output is fixed and independent of the thread count.
 *
 * Layout: every matrix is row-major; X is m x n with leading dimension ldx >= n; n x n
 * matrices are dense with leading dimension n.
 *
 * Parity status of each function is listed in its comment; every function is pinned by a
 * CPU test except the FP32-first Gram emulation, whose shift rule is not in the paper
 * (parity unpinned beyond its error bound).  In the drivers, whether a borderline unshifted
 * Cholesky breaks down (kappa near 1/u, or a factor with kappa above u^{-1/2}) depends on the
 * rounding order, so the pass count there is parity unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_U 1.1102230246251565e-16   /* 2^-53, unit roundoff of binary64 (Section 6) */
#define ORC_U32 5.9604644775390625e-08 /* 2^-24, unit roundoff of binary32 */

enum { ORC_OK = 0, ORC_BREAKDOWN = 5, ORC_NOT_CONVERGED = 6, ORC_NONFINITE = 7, ORC_INVALID = 1 };
enum { ORC_FIXED3 = 0, ORC_ADAPTIVE = 1, ORC_CHOLQR2 = 2, ORC_ITERATED = 3 };
enum { ORC_SHIFT_PAPER = 0, ORC_SHIFT_FRO = 1, ORC_SHIFT_SMALL = 2, ORC_SHIFT_CUSTOM = 3, ORC_SHIFT_DEPTH = 4 };
enum { ORC_B_NONE = 0, ORC_B_TRIDIAG = 1, ORC_B_DENSE = 2, ORC_B_CSR = 3 };

/* ------------------------------------------------------------------------------------------
 * Gram matrices (equation (eq:gram); oblique form X^T B X of Section 5, Algorithm 4).
 * a_ij = sum_k x_ki * x_kj, summed recursively over k = 0..m-1 in row order (the gamma_m
 * model of Section 3.1.1).  Only i <= j is computed; the lower triangle is a mirror.
 * Threads own disjoint sets of Gram rows i; each thread streams all of X once.
 * ---------------------------------------------------------------------------------------- */
static void owner_columns(int64_t n, int nthreads, int t, int64_t *cols, int64_t *ncols)
{
    /* Gram row i costs n - i; deal rows out in pairs (i, n-1-i) round-robin so that threads
     * get near-equal work.  The assignment changes only which thread computes an entry. */
    int64_t c = 0, k = 0;
    for (int64_t lo = 0, hi = n - 1; lo <= hi; ++lo, --hi, ++k) {
        if (k % nthreads == t) {
            cols[c++] = lo;
            if (hi != lo) cols[c++] = hi;
        }
    }
    *ncols = c;
}

/* Generic Gram driver: Y is either X itself (Euclidean) or a row-wise operator applied to X
 * by `yrow` (oblique).  Accumulators acc[i][j] for owned rows i. */
typedef void (*yrow_fn)(int64_t k, int64_t n, const double *X, int64_t ldx, int64_t m,
                        const void *ctx, double *y);

static void gram_driver(int64_t m, int64_t n, const double *X, int64_t ldx, yrow_fn yf,
                        const void *ctx, double *A)
{
#pragma omp parallel
    {
        int nt = 1, t = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t nc = 0;
        owner_columns(n, nt, t, cols, &nc);
        double *acc = (double *)calloc((size_t)(nc * n + 1), sizeof(double));
        double *y = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t k = 0; k < m; ++k) {
            const double *xk = X + k * ldx;
            const double *yk = xk;
            if (yf) {
                yf(k, n, X, ldx, m, ctx, y);
                yk = y;
            }
            for (int64_t c = 0; c < nc; ++c) {
                const int64_t i = cols[c];
                const double xi = xk[i];
                double *row = acc + c * n;
                for (int64_t j = i; j < n; ++j) row[j] = row[j] + xi * yk[j];
            }
        }
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t i = cols[c];
            for (int64_t j = i; j < n; ++j) {
                A[i * n + j] = acc[c * n + j];
                A[j * n + i] = acc[c * n + j];
            }
        }
        free(y);
        free(acc);
        free(cols);
    }
}

/* A = X^T X  (equation (eq:gram), Algorithm 1 line 1). */
void orc_gram(int64_t m, int64_t n, const double *X, int64_t ldx, double *A)
{
    gram_driver(m, n, X, ldx, NULL, NULL, A);
}

/* Tridiagonal B: (B x)_k = off_{k-1} x_{k-1} + diag_k x_k + off_k x_{k+1}, evaluated left to
 * right; missing neighbours at the ends are absent. */
typedef struct { const double *diag, *off; } tri_ctx;

static void tri_row(int64_t k, int64_t n, const double *X, int64_t ldx, int64_t m,
                    const void *vctx, double *y)
{
    const tri_ctx *c = (const tri_ctx *)vctx;
    const double *xk = X + k * ldx;
    for (int64_t j = 0; j < n; ++j) {
        double v;
        if (k > 0)
            v = c->off[k - 1] * X[(k - 1) * ldx + j] + c->diag[k] * xk[j];
        else
            v = c->diag[k] * xk[j];
        if (k + 1 < m) v = v + c->off[k] * X[(k + 1) * ldx + j];
        y[j] = v;
    }
}

/* A = X^T B X with B symmetric tridiagonal (Algorithm 4 line 1, Section 5). */
void orc_gram_tridiag(int64_t m, int64_t n, const double *X, int64_t ldx, const double *diag,
                      const double *off, double *A)
{
    tri_ctx c = {diag, off};
    gram_driver(m, n, X, ldx, tri_row, &c, A);
}

/* General sparse symmetric B in compressed sparse row form (the storage of the sparse B of
 * Section 7): (B x)_k is the sum over the stored entries e of row k, in storage order, of
 * val_e x_{col_e}, added left to right from zero. */
typedef struct {
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
} csr_ctx;

static void csr_row(int64_t k, int64_t n, const double *X, int64_t ldx, int64_t m, const void *vctx,
                    double *y)
{
    const csr_ctx *c = (const csr_ctx *)vctx;
    (void)m;
    for (int64_t j = 0; j < n; ++j) y[j] = 0.0;
    for (int64_t e = c->row_ptr[k]; e < c->row_ptr[k + 1]; ++e) {
        const double b = c->val[e];
        const double *xr = X + (int64_t)c->col[e] * ldx;
        for (int64_t j = 0; j < n; ++j) y[j] = y[j] + b * xr[j];
    }
}

/* A = X^T B X with B in compressed sparse row form (Section 7, oblique inner product; the
 * row-by-row product Y = B X followed by X^T Y, without storing Y). */
void orc_gram_csr(int64_t m, int64_t n, const double *X, int64_t ldx, const int64_t *row_ptr,
                  const int32_t *col, const double *val, double *A)
{
    csr_ctx c = {row_ptr, col, val};
    gram_driver(m, n, X, ldx, csr_row, &c, A);
}

/* A = X^T B X with dense B (m x m row-major): Y = B X by plain loops, then X^T Y. */
void orc_gram_dense(int64_t m, int64_t n, const double *X, int64_t ldx, const double *B,
                    double *A)
{
    double *Y = (double *)malloc(sizeof(double) * (size_t)(m * n));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t l = 0; l < m; ++l) v = v + B[k * m + l] * X[l * ldx + j];
            Y[k * n + j] = v;
        }
    /* a_ij = sum_k x_ki y_kj in row order, i <= j, mirrored. */
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            double v = 0.0;
            for (int64_t k = 0; k < m; ++k) v = v + X[k * ldx + i] * Y[k * n + j];
            A[i * n + j] = v;
            A[j * n + i] = v;
        }
    free(Y);
}

/* FP32-first Gram (not in the paper): every x is rounded to binary32, products are formed
 * exactly and accumulated in binary32 with one rounding per step (fmaf) over consecutive
 * chains of `chain` rows; the chain sums are added in binary64 in chain order. */
void orc_gram_f32(int64_t m, int64_t n, const double *X, int64_t ldx, int64_t chain, double *A)
{
    if (chain < 1) chain = 1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) {
        double *tot = (double *)calloc((size_t)n, sizeof(double));
        float *part = (float *)calloc((size_t)n, sizeof(float));
        for (int64_t k0 = 0; k0 < m; k0 += chain) {
            const int64_t k1 = (k0 + chain < m) ? k0 + chain : m;
            for (int64_t j = i; j < n; ++j) part[j] = 0.0f;
            for (int64_t k = k0; k < k1; ++k) {
                const float xi = (float)X[k * ldx + i];
                for (int64_t j = i; j < n; ++j) part[j] = fmaf(xi, (float)X[k * ldx + j], part[j]);
            }
            for (int64_t j = i; j < n; ++j) tot[j] = tot[j] + (double)part[j];
        }
        for (int64_t j = i; j < n; ++j) {
            A[i * n + j] = tot[j];
            A[j * n + i] = tot[j];
        }
        free(part);
        free(tot);
    }
}

/* A = X^T X with the rows summed in consecutive chunks of `chunk` rows: each chunk's products
 * are added in row order starting from zero, and the chunk sums are added in chunk order.  Every
 * product then takes part in at most orc_gram_depth(m, chunk) roundings (its own, the additions
 * inside its chunk, the additions of the chunk sums), which is the depth that replaces m in the
 * gamma_m bound of the Gram error (Section 3.1.1) for this summation order. */
void orc_gram_chunked(int64_t m, int64_t n, const double *X, int64_t ldx, int64_t chunk, double *A)
{
    if (chunk < 1) chunk = 1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) {
        double *tot = (double *)calloc((size_t)n, sizeof(double));
        double *part = (double *)calloc((size_t)n, sizeof(double));
        for (int64_t k0 = 0; k0 < m; k0 += chunk) {
            const int64_t k1 = (k0 + chunk < m) ? k0 + chunk : m;
            for (int64_t j = i; j < n; ++j) part[j] = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                const double xi = X[k * ldx + i];
                for (int64_t j = i; j < n; ++j) part[j] = part[j] + xi * X[k * ldx + j];
            }
            for (int64_t j = i; j < n; ++j) tot[j] = tot[j] + part[j];
        }
        for (int64_t j = i; j < n; ++j) {
            A[i * n + j] = tot[j];
            A[j * n + i] = tot[j];
        }
        free(part);
        free(tot);
    }
}

/* Summation depth of orc_gram_chunked: chunk + ceil(m / chunk) (m itself bounds the depth of
 * the row-order recursive sum of orc_gram). */
int64_t orc_gram_depth(int64_t m, int64_t chunk)
{
    if (chunk < 1) chunk = 1;
    if (chunk >= m) return m;
    return chunk + (m + chunk - 1) / chunk;
}

/* ------------------------------------------------------------------------------------------
 * Symmetric eigenvalues by the cyclic Jacobi method (rotations that annihilate a_pq one at a
 * time, sweeping all p < q until the off-diagonal part is negligible).  Used for ||X||_2^2 =
 * lambda_max(X^T X), the quantity the shift of equation (eq:finds2) is built from.
 * ---------------------------------------------------------------------------------------- */
void orc_sym_eig(int64_t n, const double *A, double *w)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)(n * n));
    memcpy(a, A, sizeof(double) * (size_t)(n * n));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            dia = dia + a[p * n + p] * a[p * n + p];
            for (int64_t q = p + 1; q < n; ++q) off = off + a[p * n + q] * a[p * n + q];
        }
        if (off <= 1e-36 * dia || off == 0.0) break;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                if (apq == 0.0) continue;
                const double app = a[p * n + p], aqq = a[q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int64_t k = 0; k < n; ++k) { /* columns p, q */
                    const double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) { /* rows p, q */
                    const double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                a[p * n + q] = 0.0;
                a[q * n + p] = 0.0;
            }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = a[i * n + i];
    /* insertion sort, ascending */
    for (int64_t i = 1; i < n; ++i) {
        const double v = w[i];
        int64_t j = i - 1;
        while (j >= 0 && w[j] > v) {
            w[j + 1] = w[j];
            --j;
        }
        w[j + 1] = v;
    }
    free(a);
}

double orc_lambda_max(int64_t n, const double *A)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    orc_sym_eig(n, A, w);
    const double v = w[n - 1];
    free(w);
    return v;
}

/* ------------------------------------------------------------------------------------------
 * Cholesky factorization R^T R = A + s I, R upper triangular with positive diagonal
 * (Algorithm 1 line 3).  Row j of R: the pivot radicand d = (a_jj + s) - sum_{k<j} r_kj^2;
 * breakdown when d <= 0 or d is not finite (the meaning of "chol breaks down" in Algorithm 2;
 * the same event as LAPACK potrf's info > 0).  Returns 0, or 1 + the column that broke down.
 * ---------------------------------------------------------------------------------------- */
int orc_chol_upper(int64_t n, const double *A, double s, double *R)
{
    memset(R, 0, sizeof(double) * (size_t)(n * n));
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j] + s;
        for (int64_t k = 0; k < j; ++k) d = d - R[k * n + j] * R[k * n + j];
        if (!(d > 0.0) || !isfinite(d)) return (int)(j + 1);
        const double rjj = sqrt(d);
        R[j * n + j] = rjj;
        for (int64_t l = j + 1; l < n; ++l) {
            double v = A[j * n + l];
            for (int64_t k = 0; k < j; ++k) v = v - R[k * n + j] * R[k * n + l];
            R[j * n + l] = v / rjj;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Q = X R^{-1} row by row (Algorithm 1 line 4): q_i^T R = x_i^T is solved by forward
 * substitution, q_ij = (x_ij - sum_{k<j} q_ik r_kj) / r_jj, the row-wise solve whose backward
 * error model is equation (eq:backward2).  Q may alias X (same ld).
 * ---------------------------------------------------------------------------------------- */
void orc_trsm_rows(int64_t m, int64_t n, const double *X, int64_t ldx, const double *R,
                   double *Q, int64_t ldq)
{
#pragma omp parallel
    {
        double *t = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            const double *x = X + i * ldx;
            for (int64_t j = 0; j < n; ++j) t[j] = x[j];
            /* Column sweep: once q_k is known it is removed from every later entry, so entry
             * j sees x_ij - q_i0 r_0j - q_i1 r_1j - ... in that order before its division. */
            for (int64_t k = 0; k < n; ++k) {
                const double qk = t[k] / R[k * n + k];
                t[k] = qk;
                for (int64_t j = k + 1; j < n; ++j) t[j] = t[j] - qk * R[k * n + j];
            }
            double *q = Q + i * ldq;
            for (int64_t j = 0; j < n; ++j) q[j] = t[j];
        }
        free(t);
    }
}

/* out = Rt * R for upper triangular Rt, R (the accumulation R := R~ R of Algorithms 2, 3). */
void orc_trmm_upper(int64_t n, const double *Rt, const double *R, double *out)
{
    double *o = (double *)calloc((size_t)(n * n), sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            double v = 0.0;
            for (int64_t k = i; k <= j; ++k) v = v + Rt[i * n + k] * R[k * n + j];
            o[i * n + j] = v;
        }
    memcpy(out, o, sizeof(double) * (size_t)(n * n));
    free(o);
}

/* ||B||_2 bound for tridiagonal B: max_k |off_{k-1}| + |diag_k| + |off_k| (Gershgorin; an
 * upper bound on ||B||_2 for symmetric B).  The paper leaves the estimator open. */
double orc_gershgorin_tridiag(int64_t m, const double *diag, const double *off)
{
    double best = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        double v = (k > 0 ? fabs(off[k - 1]) : 0.0) + fabs(diag[k]);
        if (k + 1 < m) v = v + fabs(off[k]);
        if (v > best) best = v;
    }
    return best;
}

/* ||B||_2 bound for B in compressed sparse row form: the largest absolute row sum, each row
 * summed in storage order (Gershgorin, as for the tridiagonal B). */
double orc_gershgorin_csr(int64_t m, const int64_t *row_ptr, const double *val)
{
    double best = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        double v = 0.0;
        for (int64_t e = row_ptr[k]; e < row_ptr[k + 1]; ++e) v = v + fabs(val[e]);
        if (v > best) best = v;
    }
    return best;
}

/* Shift of the first pass.
 *   Euclidean, equation (eq:finds2):  s = 11 (m n + n (n+1)) u ||X||_2^2
 *   Oblique,   equation (eq:finds2B): s = 11 (2 m sqrt(m n) + n (n+1)) u ||X||_2^2 ||B||_2
 *   SMALL (remark after Table 3):     s = u ||X||_2^2 (||B||_2)
 *   CUSTOM:                            s = alpha ||X||_2^2 (||B||_2)
 * `norm2sq` is ||X||_2^2 (or its Frobenius replacement); bnorm is 1 when B = I. */
double orc_shift(int64_t m, int64_t n, double norm2sq, double bnorm, int oblique, int mode,
                 double alpha)
{
    const double dm = (double)m, dn = (double)n;
    double c;
    if (mode == ORC_SHIFT_SMALL)
        c = ORC_U;
    else if (mode == ORC_SHIFT_CUSTOM)
        c = alpha;
    else if (oblique)
        c = 11.0 * (2.0 * dm * sqrt(dm * dn) + dn * (dn + 1.0)) * ORC_U;
    else
        c = 11.0 * (dm * dn + dn * (dn + 1.0)) * ORC_U;
    return c * norm2sq * bnorm;
}

/* Summation-depth shift (the shift-policy question the paper leaves open in its remark after
 * Table 3 and its conclusion): the derivation of equation (eq:finds2) with gamma_m, the bound of a
 * Gram summed over m rows in sequence, replaced by gamma_d for a Gram whose sums have depth d:
 *   s = 11 (d n + n (n+1)) u ||X||_2^2;  d = m gives equation (eq:finds2). */
double orc_shift_depth(int64_t depth, int64_t n, double norm2sq)
{
    const double dd = (double)depth, dn = (double)n;
    return 11.0 * (dd * dn + dn * (dn + 1.0)) * ORC_U * norm2sq;
}

/* Shift of an FP32-first pass (not in the paper): the Gram error of a binary32 chain of
 * `chain` rows plus the rounding of X to binary32 is bounded like gamma_{chain+2} in u32,
 * and the Cholesky itself runs in binary64:
 *   s32 = 11 ((chain + 2) n u32 + n (n+1) u) ||X||_2^2. */
double orc_shift_f32(int64_t n, int64_t chain, double norm2sq)
{
    const double dn = (double)n;
    return 11.0 * (((double)chain + 2.0) * dn * ORC_U32 + dn * (dn + 1.0) * ORC_U) * norm2sq;
}

/* ------------------------------------------------------------------------------------------
 * Driver: Algorithm 3 (shiftedCholeskyQR3), Algorithm 2 (iterated, shift on breakdown),
 * CholeskyQR2, and "Algorithm 3 with Algorithm 2 continuation" (ADAPTIVE).
 *
 * Readings where the paper is silent or inconsistent (each listed in the design notes):
 *  - Algorithm 3's fifth step applies the R just computed by the shifted Cholesky.
 *  - Algorithm 5's CholeskyQR2 steps use the B-Gram Q^T B Q.
 *  - A shift after pass 1 uses the largest eigenvalue of the current Gram (||Q||_2^2 of the
 *    current iterate) in place of ||X||_2^2; in the oblique case that Gram is Q^T B Q, its
 *    largest eigenvalue stands for ||Q||_2^2 ||B||_2, and the constant of (eq:finds2B) stays.
 *  - Algorithm 2's stopping test ||Q^T Q - I||_F <= sqrt(n) u is replaced by: a pass is the
 *    last one when it ran unshifted and its input Gram had ||A - I||_F <= 1/2.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int32_t schedule;            /* ORC_FIXED3 / ADAPTIVE / CHOLQR2 / ITERATED */
    int32_t shift_mode;          /* ORC_SHIFT_* */
    int32_t max_passes;          /* adaptive cap (<= 16) */
    int32_t precision;           /* 0 FP64, 1 FP32-first */
    int32_t f32_chain;           /* rows per binary32 chain for FP32-first */
    int32_t force_breakdown_pass; /* debug: the Cholesky of this pass (1-based) reports breakdown */
    int32_t zero_shift;          /* debug: every shift is 0 */
    int32_t gram_chunk;          /* ORC_SHIFT_DEPTH: rows per chunk of every Gram */
    double custom_alpha;
    double bnorm;                /* >0: ||B||_2 bound given by caller */
} orc_opts;

typedef struct {
    int32_t status, passes, shifted_mask, breakdown_mask, fell_back, pad;
    double shift[16];
    double norm2sq[16];
    double gram_dev[16]; /* ||A_p - I||_F of the input Gram of each pass */
} orc_info;

static int all_finite(int64_t k, const double *v)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static double dev_from_identity(int64_t n, const double *A)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const double d = A[i * n + j] - (i == j ? 1.0 : 0.0);
            s = s + d * d;
        }
    return sqrt(s);
}

/* B descriptor: kind 0 none, 1 tridiagonal (diag[m], off[m-1]), 2 dense (m x m), 3 compressed
 * sparse rows (row_ptr[m+1], col[nnz], val[nnz]). */
typedef struct {
    int32_t kind;
    const double *b0, *b1;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
} bop_t;

static int scqr_run(int64_t m, int64_t n, const double *X, int64_t ldx, const bop_t *bop,
                    const orc_opts *opt, double *Q, double *R, orc_info *info, double *gram_hist,
                    double *rt_hist)
{
    const int32_t bkind = bop->kind;
    const double *b0 = bop->b0, *b1 = bop->b1;
    memset(info, 0, sizeof(*info));
    const int depth_mode = opt->shift_mode == ORC_SHIFT_DEPTH;
    if (m < n || n < 1 || ldx < n || opt->max_passes < 1 || opt->max_passes > 16 ||
        (depth_mode && (bkind != ORC_B_NONE || opt->gram_chunk < 1))) {
        info->status = ORC_INVALID;
        return ORC_INVALID;
    }
    const int64_t nn = n * n;
    double *A = (double *)malloc(sizeof(double) * (size_t)nn);
    double *Ae = (double *)malloc(sizeof(double) * (size_t)nn);
    double *Rt = (double *)malloc(sizeof(double) * (size_t)nn);
    const int oblique = bkind != ORC_B_NONE;
    double bnorm = 1.0;
    if (oblique) {
        if (opt->bnorm > 0.0)
            bnorm = opt->bnorm;
        else if (bkind == ORC_B_TRIDIAG)
            bnorm = orc_gershgorin_tridiag(m, b0, b1);
        else if (bkind == ORC_B_CSR)
            bnorm = orc_gershgorin_csr(m, bop->row_ptr, bop->val);
        else {
            double *w = (double *)malloc(sizeof(double) * (size_t)(m));
            orc_sym_eig(m, b0, w);
            bnorm = w[m - 1];
            free(w);
        }
    }
    int max_p = opt->max_passes;
    if (opt->schedule == ORC_FIXED3) max_p = 3;
    if (opt->schedule == ORC_CHOLQR2) max_p = 2;

    for (int64_t i = 0; i < m; ++i) memcpy(Q + i * n, X + i * ldx, sizeof(double) * (size_t)n);
    memset(R, 0, sizeof(double) * (size_t)nn);
    for (int64_t i = 0; i < n; ++i) R[i * n + i] = 1.0;

    int status = ORC_NOT_CONVERGED;
    int passes = 0;
    for (int p = 1; p <= max_p; ++p) {
        const int first = (p == 1);
        int f32 = first && opt->precision == 1 && !oblique;
        /* Gram of the current iterate (Algorithm 2 line 3; Algorithm 3 lines 2, 6, 7). */
        if (f32) {
            orc_gram_f32(m, n, Q, n, opt->f32_chain, A);
            if (!all_finite(nn, A)) {
                /* the binary32 Gram overflowed (or X holds a NaN / Inf): the first pass is
                 * redone in binary64, whose own finiteness test decides the status */
                info->fell_back = 1;
                f32 = 0;
                orc_gram(m, n, Q, n, A);
            }
        } else if (bkind == ORC_B_TRIDIAG)
            orc_gram_tridiag(m, n, Q, n, b0, b1, A);
        else if (bkind == ORC_B_DENSE)
            orc_gram_dense(m, n, Q, n, b0, A);
        else if (bkind == ORC_B_CSR)
            orc_gram_csr(m, n, Q, n, bop->row_ptr, bop->col, bop->val, A);
        else if (depth_mode)
            orc_gram_chunked(m, n, Q, n, opt->gram_chunk, A);
        else
            orc_gram(m, n, Q, n, A);
        if (!all_finite(nn, A)) {
            status = ORC_NONFINITE;
            passes = p - 1;
            break;
        }
        info->gram_dev[p - 1] = dev_from_identity(n, A);
        if (gram_hist) memcpy(gram_hist + (p - 1) * nn, A, sizeof(double) * (size_t)nn);

        /* Norm used by a shift of this pass. */
        double norm2sq;
        if (first && oblique) {
            orc_gram(m, n, Q, n, Ae); /* ||X||_2 of equation (eq:finds2B) is Euclidean */
            norm2sq = 0.0;
            if (opt->shift_mode == ORC_SHIFT_FRO)
                for (int64_t i = 0; i < n; ++i) norm2sq = norm2sq + Ae[i * n + i];
            else
                norm2sq = orc_lambda_max(n, Ae);
        } else if (opt->shift_mode == ORC_SHIFT_FRO) {
            norm2sq = 0.0;
            for (int64_t i = 0; i < n; ++i) norm2sq = norm2sq + A[i * n + i];
        } else {
            norm2sq = orc_lambda_max(n, A);
        }
        const double bfac = (first && oblique) ? bnorm : 1.0;
        info->norm2sq[p - 1] = norm2sq;
        const double s_pass = depth_mode ? orc_shift_depth(orc_gram_depth(m, opt->gram_chunk), n, norm2sq)
                                         : orc_shift(m, n, norm2sq, bfac, oblique, opt->shift_mode,
                                                     opt->custom_alpha);

        const int forced = (opt->force_breakdown_pass == p);
        const int shift_first = first && (opt->schedule == ORC_FIXED3 || opt->schedule == ORC_ADAPTIVE);
        int shifted = 0, bd;
        double s = 0.0;
        if (shift_first) {
            if (f32) {
                s = orc_shift_f32(n, opt->f32_chain, norm2sq);
                if (s > 0.01 * norm2sq || (bd = (forced ? 1 : orc_chol_upper(n, A, opt->zero_shift ? 0.0 : s, Rt))) != 0) {
                    /* Fallback to the binary64 pass. */
                    info->fell_back = 1;
                    orc_gram(m, n, Q, n, A);
                    info->gram_dev[0] = dev_from_identity(n, A);
                    if (gram_hist) memcpy(gram_hist, A, sizeof(double) * (size_t)nn);
                    norm2sq = (opt->shift_mode == ORC_SHIFT_FRO) ? 0.0 : orc_lambda_max(n, A);
                    if (opt->shift_mode == ORC_SHIFT_FRO)
                        for (int64_t i = 0; i < n; ++i) norm2sq = norm2sq + A[i * n + i];
                    info->norm2sq[0] = norm2sq;
                    s = orc_shift(m, n, norm2sq, 1.0, 0, opt->shift_mode, opt->custom_alpha);
                    if (opt->zero_shift) s = 0.0;
                    bd = orc_chol_upper(n, A, s, Rt);
                }
            } else {
                s = s_pass;
                if (opt->zero_shift) s = 0.0;
                bd = forced ? 1 : orc_chol_upper(n, A, s, Rt);
            }
            shifted = 1;
            info->shift[p - 1] = s;
            if (bd) {
                info->shifted_mask |= 1 << (p - 1);
                info->breakdown_mask |= 1 << (p - 1);
                status = ORC_BREAKDOWN;
                passes = p - 1;
                break;
            }
        } else {
            bd = forced ? 1 : orc_chol_upper(n, A, 0.0, Rt);
            if (bd) {
                info->breakdown_mask |= 1 << (p - 1);
                if (opt->schedule == ORC_ADAPTIVE || opt->schedule == ORC_ITERATED) {
                    s = s_pass;
                    if (opt->zero_shift) s = 0.0;
                    shifted = 1;
                    info->shift[p - 1] = s;
                    info->shifted_mask |= 1 << (p - 1);
                    bd = orc_chol_upper(n, A, s, Rt);
                }
                if (bd) {
                    status = ORC_BREAKDOWN;
                    passes = p - 1;
                    break;
                }
            }
        }
        if (shifted) info->shifted_mask |= 1 << (p - 1);
        info->shift[p - 1] = s;
        if (rt_hist) memcpy(rt_hist + (p - 1) * nn, Rt, sizeof(double) * (size_t)nn);

        /* Q := Q R~^{-1}, R := R~ R */
        orc_trsm_rows(m, n, Q, n, Rt, Q, n);
        orc_trmm_upper(n, Rt, R, R);
        passes = p;

        int last;
        if (opt->schedule == ORC_FIXED3)
            last = (p == 3);
        else if (opt->schedule == ORC_CHOLQR2)
            last = (p == 2);
        else
            last = (!shifted && info->gram_dev[p - 1] <= 0.5);
        if (last) {
            status = ORC_OK;
            break;
        }
    }
    info->status = status;
    info->passes = passes;
    free(Rt);
    free(Ae);
    free(A);
    return status;
}

int orc_scqr(int64_t m, int64_t n, const double *X, int64_t ldx, int32_t bkind, const double *b0,
             const double *b1, const orc_opts *opt, double *Q, double *R, orc_info *info,
             double *gram_hist, double *rt_hist)
{
    if (bkind == ORC_B_CSR) {
        memset(info, 0, sizeof(*info));
        info->status = ORC_INVALID;
        return ORC_INVALID;
    }
    const bop_t b = {bkind, b0, b1, NULL, NULL, NULL};
    return scqr_run(m, n, X, ldx, &b, opt, Q, R, info, gram_hist, rt_hist);
}

/* The driver with B in compressed sparse row form (Section 7). */
int orc_scqr_csr(int64_t m, int64_t n, const double *X, int64_t ldx, const int64_t *row_ptr,
                 const int32_t *col, const double *val, const orc_opts *opt, double *Q, double *R,
                 orc_info *info, double *gram_hist, double *rt_hist)
{
    const bop_t b = {ORC_B_CSR, NULL, NULL, row_ptr, col, val};
    return scqr_run(m, n, X, ldx, &b, opt, Q, R, info, gram_hist, rt_hist);
}

/* ------------------------------------------------------------------------------------------
 * QR adjoint (not in the paper): for X = QR (thin, R upper with positive diagonal) and
 * upstream gradients dQ, dR (only the upper triangle of dR is read):
 *   G = dQ^T Q,  M = R dR^T - G,  C = copyltu(M) (C_ij = M_{max(i,j), min(i,j)}),
 *   dX = (dQ + Q C) R^{-T}, solved row by row: dX R^T = Y by back substitution.
 * dQ or dR may be NULL (treated as zero).
 * ---------------------------------------------------------------------------------------- */
void orc_qr_backward(int64_t m, int64_t n, const double *Q, const double *R, const double *dQ,
                     const double *dR, double *dX)
{
    const int64_t nn = n * n;
    double *G = (double *)calloc((size_t)nn, sizeof(double));
    double *M = (double *)calloc((size_t)nn, sizeof(double));
    double *C = (double *)calloc((size_t)nn, sizeof(double));
    if (dQ) {
        /* G_ij = sum_k dQ_ki Q_kj, row order, every (i, j). */
#pragma omp parallel for schedule(dynamic)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double v = 0.0;
                for (int64_t k = 0; k < m; ++k) v = v + dQ[k * n + i] * Q[k * n + j];
                G[i * n + j] = v;
            }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            if (dR) {
                /* (R dR^T)_ij = sum_k R_ik dR_jk, nonzero for k >= max(i, j) */
                const int64_t k0 = i > j ? i : j;
                for (int64_t k = k0; k < n; ++k) v = v + R[i * n + k] * dR[j * n + k];
            }
            M[i * n + j] = v - G[i * n + j];
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) C[i * n + j] = (i >= j) ? M[i * n + j] : M[j * n + i];
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < m; ++r) {
            const double *q = Q + r * n;
            for (int64_t j = 0; j < n; ++j) {
                double v = 0.0;
                for (int64_t k = 0; k < n; ++k) v = v + q[k] * C[k * n + j];
                y[j] = (dQ ? dQ[r * n + j] : 0.0) + v;
            }
            double *dx = dX + r * n;
            for (int64_t j = n - 1; j >= 0; --j) {
                double v = y[j];
                for (int64_t k = j + 1; k < n; ++k) v = v - dx[k] * R[j * n + k];
                dx[j] = v / R[j * n + j];
            }
        }
        free(y);
    }
    free(C);
    free(M);
    free(G);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
