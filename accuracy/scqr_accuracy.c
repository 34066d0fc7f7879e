/*
 * Accuracy measurements for a computed QR factorization X ~ Q R (CPU, binary64).
 *
 * Measuring ||Q^T Q - I|| at the level of the unit roundoff for tall Q needs a Gram that is
 * more accurate than plain recursive summation (whose error grows like m u for m rows), so
 * every inner product here is compensated: Dot2 of Ogita, Rump and Oishi (error-free
 * TwoProduct through fma, TwoSum for the running sum), which is as accurate as evaluating
 * in twice the working precision and rounding once.
 *
 * Independent of the oracle and of the GPU library; shares no code with either.
 * Row-major layouts, leading dimensions given explicitly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double hi, lo;
} dd;

static inline void two_sum(double a, double b, double *s, double *e)
{
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* acc += a * b, compensated */
static inline void dot2_step(dd *acc, double a, double b)
{
    const double p = a * b;
    const double pe = fma(a, b, -p);
    double s, se;
    two_sum(acc->hi, p, &s, &se);
    acc->hi = s;
    acc->lo = acc->lo + (se + pe);
}

/* acc += a * b * c with the product formed to double-double accuracy */
static inline void dot2_step3(dd *acc, double a, double b, double c)
{
    const double p = a * b;
    const double pe = fma(a, b, -p);
    const double q = p * c;
    const double qe = fma(p, c, -q);
    double s, se;
    two_sum(acc->hi, q, &s, &se);
    acc->hi = s;
    acc->lo = acc->lo + (se + qe + pe * c);
}

/* G = Q^T Q (full symmetric n x n), every entry a compensated dot product. */
void acc_gram_dot2(int64_t m, int64_t n, const double *Q, int64_t ldq, double *G)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) {
        dd *acc = (dd *)calloc((size_t)n, sizeof(dd));
        for (int64_t k = 0; k < m; ++k) {
            const double *q = Q + k * ldq;
            const double qi = q[i];
            for (int64_t j = i; j < n; ++j) dot2_step(&acc[j], qi, q[j]);
        }
        for (int64_t j = i; j < n; ++j) {
            const double v = acc[j].hi + acc[j].lo;
            G[i * n + j] = v;
            G[j * n + i] = v;
        }
        free(acc);
    }
}

/* G = Q^T B Q for symmetric tridiagonal B (diag[m], off[m-1]), compensated. */
void acc_gram_dot2_tridiag(int64_t m, int64_t n, const double *Q, int64_t ldq,
                           const double *diag, const double *off, double *G)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) {
        dd *acc = (dd *)calloc((size_t)n, sizeof(dd));
        for (int64_t k = 0; k < m; ++k) {
            const double *q = Q + k * ldq;
            const double qi = q[i];
            for (int64_t j = i; j < n; ++j) {
                dot2_step3(&acc[j], qi, q[j], diag[k]);
                if (k > 0) dot2_step3(&acc[j], qi, Q[(k - 1) * ldq + j], off[k - 1]);
                if (k + 1 < m) dot2_step3(&acc[j], qi, Q[(k + 1) * ldq + j], off[k]);
            }
        }
        for (int64_t j = i; j < n; ++j) {
            const double v = acc[j].hi + acc[j].lo;
            G[i * n + j] = v;
            G[j * n + i] = v;
        }
        free(acc);
    }
}

/* G = Q^T B Q for symmetric B in compressed sparse row form (row_ptr[m+1], col, val),
 * compensated: every term q_ki * val_e * q_{col_e, j} enters one double-double sum. */
void acc_gram_dot2_csr(int64_t m, int64_t n, const double *Q, int64_t ldq, const int64_t *row_ptr,
                       const int32_t *col, const double *val, double *G)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) {
        dd *acc = (dd *)calloc((size_t)n, sizeof(dd));
        for (int64_t k = 0; k < m; ++k) {
            const double qi = Q[k * ldq + i];
            for (int64_t e = row_ptr[k]; e < row_ptr[k + 1]; ++e) {
                const double *qc = Q + (int64_t)col[e] * ldq;
                const double b = val[e];
                for (int64_t j = i; j < n; ++j) dot2_step3(&acc[j], qi, qc[j], b);
            }
        }
        for (int64_t j = i; j < n; ++j) {
            const double v = acc[j].hi + acc[j].lo;
            G[i * n + j] = v;
            G[j * n + i] = v;
        }
        free(acc);
    }
}

/* Returns ||X - Q R||_F and writes ||X||_F to *xnorm.  R is n x n upper triangular
 * (only the upper triangle is read).  Each entry of Q R is a compensated dot product and the
 * squares are accumulated compensated per row, then per thread, then in thread order of
 * fixed row blocks (deterministic for a given thread count up to the final double add). */
double acc_residual(int64_t m, int64_t n, const double *X, int64_t ldx, const double *Q,
                    int64_t ldq, const double *R, int64_t ldr, double *xnorm)
{
    const int64_t nblk = 256;
    double *res = (double *)calloc((size_t)nblk, sizeof(double));
    double *xs = (double *)calloc((size_t)nblk, sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t r0 = m * b / nblk, r1 = m * (b + 1) / nblk;
        dd e2 = {0.0, 0.0}, x2 = {0.0, 0.0};
        for (int64_t r = r0; r < r1; ++r) {
            const double *q = Q + r * ldq;
            const double *x = X + r * ldx;
            for (int64_t j = 0; j < n; ++j) {
                dd acc = {0.0, 0.0};
                /* x_rj - sum_{k<=j} q_rk r_kj */
                dot2_step(&acc, x[j], 1.0);
                for (int64_t k = 0; k <= j; ++k) dot2_step(&acc, -q[k], R[k * ldr + j]);
                const double e = acc.hi + acc.lo;
                dot2_step(&e2, e, e);
                dot2_step(&x2, x[j], x[j]);
            }
        }
        res[b] = e2.hi + e2.lo;
        xs[b] = x2.hi + x2.lo;
    }
    dd te = {0.0, 0.0}, tx = {0.0, 0.0};
    for (int64_t b = 0; b < nblk; ++b) {
        dot2_step(&te, res[b], 1.0);
        dot2_step(&tx, xs[b], 1.0);
    }
    free(res);
    free(xs);
    *xnorm = sqrt(tx.hi + tx.lo);
    return sqrt(te.hi + te.lo);
}

/* Row-sampled residual: the same quantity restricted to the listed rows. */
double acc_residual_rows(int64_t nrows, const int64_t *rows, int64_t n, const double *X,
                         int64_t ldx, const double *Q, int64_t ldq, const double *R, int64_t ldr,
                         double *xnorm)
{
    dd e2 = {0.0, 0.0}, x2 = {0.0, 0.0};
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t r = rows[t];
        const double *q = Q + r * ldq;
        const double *x = X + r * ldx;
        for (int64_t j = 0; j < n; ++j) {
            dd acc = {0.0, 0.0};
            dot2_step(&acc, x[j], 1.0);
            for (int64_t k = 0; k <= j; ++k) dot2_step(&acc, -q[k], R[k * ldr + j]);
            const double e = acc.hi + acc.lo;
            dot2_step(&e2, e, e);
            dot2_step(&x2, x[j], x[j]);
        }
    }
    *xnorm = sqrt(x2.hi + x2.lo);
    return sqrt(e2.hi + e2.lo);
}
