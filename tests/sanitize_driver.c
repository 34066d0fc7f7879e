/* Host sanitizer run of the oracle and the accuracy helpers (test infrastructure only).
 *
 * Built by tests/test_sanitizers.py together with oracle/scqr_oracle.c (included below, so the
 * option and info records have the oracle's own layout) and accuracy/scqr_accuracy.c (its own
 * translation unit) under -fsanitize=address,undefined.  Every exported entry point runs on
 * small inputs: all B forms, all schedules and shift modes, the FP32-first pass, the depth
 * shift, the adjoint with and without each gradient, invalid arguments, n = 1 and m = n.  A
 * sanitizer report aborts the run; the few checks here only make sure each call did its work. */
#include <stdio.h>

#include "../oracle/scqr_oracle.c"

void acc_gram_dot2(int64_t m, int64_t n, const double *Q, int64_t ldq, double *G);
void acc_gram_dot2_tridiag(int64_t m, int64_t n, const double *Q, int64_t ldq, const double *diag,
                           const double *off, double *G);
void acc_gram_dot2_csr(int64_t m, int64_t n, const double *Q, int64_t ldq, const int64_t *row_ptr,
                       const int32_t *col, const double *val, double *G);
double acc_residual(int64_t m, int64_t n, const double *X, int64_t ldx, const double *Q, int64_t ldq,
                    const double *R, int64_t ldr, double *xnorm);
double acc_residual_rows(int64_t nrows, const int64_t *rows, int64_t n, const double *X, int64_t ldx,
                         const double *Q, int64_t ldq, const double *R, int64_t ldr, double *xnorm);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double urand(void) /* xorshift64*, uniform in [-1, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    const uint64_t r = rng_state * 0x2545f4914f6cdd1dull;
    return (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "check failed: %s\n", what);
        ++failures;
    }
}

static orc_opts opts(int schedule)
{
    orc_opts o;
    memset(&o, 0, sizeof(o));
    o.schedule = schedule;
    o.shift_mode = ORC_SHIFT_PAPER;
    o.max_passes = 8;
    o.f32_chain = 32;
    o.gram_chunk = 64;
    return o;
}

/* one factorization of an m x n X (leading dimension ldx) with B of kind bkind */
static void run_case(int64_t m, int64_t n, int64_t ldx, int32_t bkind, int schedule, int shift_mode,
                     int precision)
{
    double *X = malloc(sizeof(double) * (size_t)(m * ldx));
    for (int64_t i = 0; i < m * ldx; ++i) X[i] = urand();
    double *d = malloc(sizeof(double) * (size_t)m), *o = malloc(sizeof(double) * (size_t)m);
    for (int64_t k = 0; k < m; ++k) {
        d[k] = 4.0 + urand();
        o[k] = 0.5 * urand();
    }
    double *Bd = NULL;
    if (bkind == ORC_B_DENSE) {
        Bd = calloc((size_t)(m * m), sizeof(double));
        for (int64_t k = 0; k < m; ++k) {
            Bd[k * m + k] = d[k];
            if (k + 1 < m) Bd[k * m + k + 1] = Bd[(k + 1) * m + k] = o[k];
        }
    }
    double *Q = malloc(sizeof(double) * (size_t)(m * n)), *R = malloc(sizeof(double) * (size_t)(n * n));
    double *gh = malloc(sizeof(double) * (size_t)(16 * n * n)), *rh = malloc(sizeof(double) * (size_t)(16 * n * n));
    orc_opts op = opts(schedule);
    op.shift_mode = shift_mode;
    op.precision = precision;
    orc_info info;
    const double *b0 = bkind == ORC_B_TRIDIAG ? d : Bd, *b1 = bkind == ORC_B_TRIDIAG ? o : NULL;
    const int st = orc_scqr(m, n, X, ldx, bkind, b0, b1, &op, Q, R, &info, gh, rh);
    check(st == ORC_OK && info.passes >= 1, "orc_scqr status");
    if (bkind == ORC_B_NONE && st == ORC_OK) {
        double xn;
        const double res = acc_residual(m, n, X, ldx, Q, n, R, n, &xn);
        check(res <= 1e-12, "residual");
        const int64_t rows[3] = {0, m / 2, m - 1};
        acc_residual_rows(3, rows, n, X, ldx, Q, n, R, n, &xn);
        double *G = malloc(sizeof(double) * (size_t)(n * n));
        acc_gram_dot2(m, n, Q, n, G);
        free(G);
    }
    if (bkind == ORC_B_TRIDIAG && st == ORC_OK) {
        double *G = malloc(sizeof(double) * (size_t)(n * n));
        acc_gram_dot2_tridiag(m, n, Q, n, d, o, G);
        free(G);
    }
    free(rh);
    free(gh);
    free(R);
    free(Q);
    free(Bd);
    free(o);
    free(d);
    free(X);
}

static void csr_case(int64_t m, int64_t n)
{
    /* tridiagonal B stored as CSR, entries of row k at columns k-1, k, k+1 */
    int64_t *rp = malloc(sizeof(int64_t) * (size_t)(m + 1));
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(3 * m));
    double *val = malloc(sizeof(double) * (size_t)(3 * m));
    double *off = malloc(sizeof(double) * (size_t)m);
    for (int64_t k = 0; k < m; ++k) off[k] = 0.5 * urand();
    int64_t e = 0;
    for (int64_t k = 0; k < m; ++k) {
        rp[k] = e;
        if (k > 0) {
            col[e] = (int32_t)(k - 1);
            val[e++] = off[k - 1];
        }
        col[e] = (int32_t)k;
        val[e++] = 4.0 + urand();
        if (k + 1 < m) {
            col[e] = (int32_t)(k + 1);
            val[e++] = off[k];
        }
    }
    rp[m] = e;
    double *X = malloc(sizeof(double) * (size_t)(m * n)), *Q = malloc(sizeof(double) * (size_t)(m * n));
    double *R = malloc(sizeof(double) * (size_t)(n * n)), *G = malloc(sizeof(double) * (size_t)(n * n));
    for (int64_t i = 0; i < m * n; ++i) X[i] = urand();
    orc_gram_csr(m, n, X, n, rp, col, val, G);
    check(orc_gershgorin_csr(m, rp, val) > 0.0, "gershgorin csr");
    orc_opts op = opts(ORC_ADAPTIVE);
    orc_info info;
    check(orc_scqr_csr(m, n, X, n, rp, col, val, &op, Q, R, &info, NULL, NULL) == ORC_OK, "orc_scqr_csr");
    acc_gram_dot2_csr(m, n, Q, n, rp, col, val, G);
    /* the CSR form through orc_scqr is refused */
    check(orc_scqr(m, n, X, n, ORC_B_CSR, NULL, NULL, &op, Q, R, &info, NULL, NULL) == ORC_INVALID,
          "csr via orc_scqr");
    free(G);
    free(R);
    free(Q);
    free(X);
    free(off);
    free(val);
    free(col);
    free(rp);
}

static void kernels_case(int64_t m, int64_t n)
{
    double *X = malloc(sizeof(double) * (size_t)(m * n)), *A = malloc(sizeof(double) * (size_t)(n * n));
    double *R = malloc(sizeof(double) * (size_t)(n * n)), *P = malloc(sizeof(double) * (size_t)(n * n));
    double *Q = malloc(sizeof(double) * (size_t)(m * n)), *w = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < m * n; ++i) X[i] = urand();
    orc_gram(m, n, X, n, A);
    orc_gram_f32(m, n, X, n, 16, A);
    orc_gram_chunked(m, n, X, n, 7, A);
    check(orc_gram_depth(m, 7) >= 1, "depth");
    orc_sym_eig(n, A, w);
    check(orc_lambda_max(n, A) >= w[0], "lambda_max");
    check(orc_chol_upper(n, A, orc_shift(m, n, w[n - 1], 1.0, 0, ORC_SHIFT_PAPER, 0.0), R) == 0, "chol");
    orc_trsm_rows(m, n, X, n, R, Q, n);
    orc_trmm_upper(n, R, R, P);
    orc_shift_depth(100, n, 1.0);
    orc_shift_f32(n, 32, 1.0);
    /* the adjoint with both gradients, with dQ only and with dR only */
    double *dQ = malloc(sizeof(double) * (size_t)(m * n)), *dR = malloc(sizeof(double) * (size_t)(n * n));
    double *dX = malloc(sizeof(double) * (size_t)(m * n));
    for (int64_t i = 0; i < m * n; ++i) dQ[i] = urand();
    for (int64_t i = 0; i < n * n; ++i) dR[i] = urand();
    orc_qr_backward(m, n, Q, R, dQ, dR, dX);
    orc_qr_backward(m, n, Q, R, dQ, NULL, dX);
    orc_qr_backward(m, n, Q, R, NULL, dR, dX);
    /* a zero matrix breaks down at the first pivot */
    memset(A, 0, sizeof(double) * (size_t)(n * n));
    check(orc_chol_upper(n, A, 0.0, R) == 1, "zero pivot");
    free(dX);
    free(dR);
    free(dQ);
    free(w);
    free(Q);
    free(P);
    free(R);
    free(A);
    free(X);
}

int main(void)
{
    orc_set_num_threads(2);
    check(orc_num_threads() >= 1, "threads");
    const int schedules[4] = {ORC_FIXED3, ORC_ADAPTIVE, ORC_CHOLQR2, ORC_ITERATED};
    for (int s = 0; s < 4; ++s) run_case(300, 7, 7, ORC_B_NONE, schedules[s], ORC_SHIFT_PAPER, 0);
    run_case(257, 9, 12, ORC_B_NONE, ORC_ADAPTIVE, ORC_SHIFT_FRO, 0);     /* strided X */
    run_case(200, 5, 5, ORC_B_NONE, ORC_ADAPTIVE, ORC_SHIFT_SMALL, 0);
    run_case(300, 8, 8, ORC_B_NONE, ORC_ADAPTIVE, ORC_SHIFT_DEPTH, 0);
    run_case(300, 8, 8, ORC_B_NONE, ORC_ADAPTIVE, ORC_SHIFT_PAPER, 1);    /* FP32-first */
    run_case(300, 8, 8, ORC_B_TRIDIAG, ORC_ADAPTIVE, ORC_SHIFT_PAPER, 0);
    run_case(60, 6, 6, ORC_B_DENSE, ORC_ADAPTIVE, ORC_SHIFT_PAPER, 0);
    run_case(40, 1, 1, ORC_B_NONE, ORC_ADAPTIVE, ORC_SHIFT_PAPER, 0);     /* n = 1 */
    run_case(12, 12, 12, ORC_B_NONE, ORC_FIXED3, ORC_SHIFT_PAPER, 0);     /* m = n */
    csr_case(150, 6);
    kernels_case(90, 5);
    kernels_case(3, 1);
    /* invalid arguments are refused before any access */
    orc_opts op = opts(ORC_ADAPTIVE);
    orc_info info;
    double x[4] = {1, 2, 3, 4}, q[4], r[4];
    check(orc_scqr(1, 2, x, 2, ORC_B_NONE, NULL, NULL, &op, q, r, &info, NULL, NULL) == ORC_INVALID, "m < n");
    check(orc_scqr(2, 2, x, 1, ORC_B_NONE, NULL, NULL, &op, q, r, &info, NULL, NULL) == ORC_INVALID, "ldx < n");
    op.max_passes = 17;
    check(orc_scqr(2, 2, x, 2, ORC_B_NONE, NULL, NULL, &op, q, r, &info, NULL, NULL) == ORC_INVALID, "passes");
    if (failures) return 1;
    printf("sanitized oracle and accuracy runs: ok\n");
    return 0;
}
