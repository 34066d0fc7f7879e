// C ABI of libscqr.so: argument validation, workspace carving and the enqueue sequence of the
// shifted Cholesky QR schedules.  Every decision that depends on computed values (shift,
// breakdown, stopping test) is taken on the device by the Cholesky kernel; the host enqueues
// the longest schedule and later kernels skip themselves through the device control block.
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "scqr_internal.h"

using namespace scqr;

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- profiling
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::atomic<int> g_prof_on{0};
std::vector<ProfRec> g_prof;
thread_local hipEvent_t t_pending_a = nullptr;
thread_local const char *t_pending_name = nullptr;

}  // namespace

namespace scqr {
void prof_before(hipStream_t s, const char *name)
{
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    (void)hipEventRecord(a, s);
    t_pending_a = a;
    t_pending_name = name;
}
void prof_after(hipStream_t s)
{
    if (!g_prof_on.load(std::memory_order_relaxed) || !t_pending_a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({t_pending_name, t_pending_a, b});
    t_pending_a = nullptr;
}
}  // namespace scqr

namespace {

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

size_t mat_bytes(int64_t rows, int64_t cols, int64_t ld)
{
    if (rows <= 0) return 0;
    return sizeof(double) * (size_t)((rows - 1) * ld + cols);
}

// Bound on the summation depth of the binary64 Grams (the d of SCQR_SHIFT_DEPTH): the rows
// one accumulator chain takes (at most the rows of one workgroup: ceil(m / nwg) plus a partial
// panel round, 256 rows), the four products of one MFMA step, the fixed-order sum over the
// waves of a workgroup (at most 16) and the two reduction levels (32 partials, then nlvl2).
double gram_depth_single(int64_t m, int nwg, int nlvl2)
{
    return (double)((m + nwg - 1) / nwg + 256 + 4 + 16 + 32 + nlvl2);
}
// Batched: a task of task_rows rows is one workgroup's chain; the instance's ntask partials
// are summed in one sequence.
double gram_depth_batched(int64_t task_rows, int ntask) { return (double)(task_rows + 256 + 4 + 16 + ntask); }

scqr_status check_opts(const scqr_opts *o)
{
    if (o->schedule < 0 || o->schedule > 3) return SCQR_E_INVALID;
    if (o->shift_mode < 0 || o->shift_mode > 4) return SCQR_E_INVALID;
    if (o->precision < 0 || o->precision > 1) return SCQR_E_INVALID;
    if (o->max_passes < 1 || o->max_passes > SCQR_MAX_PASSES) return SCQR_E_INVALID;
    if (o->shift_mode == SCQR_SHIFT_CUSTOM && !(o->custom_alpha >= 0.0)) return SCQR_E_INVALID;
    if (o->recompute < 0 || o->recompute > 1) return SCQR_E_INVALID;
    return SCQR_OK;
}

struct Layout {
    int np, nwg, nlvl2;
    int64_t elems;
    size_t off_ctl, off_G, off_Ge, off_Rt, off_dinv, off_R0, off_R1, off_part, off_lvl2, off_gsum, off_bmax,
        off_vprev, off_split, total;
};

// csr: the sparse-B Gram gathers rows of X with long latencies, so it runs more workgroups
// (four per workgroup of the pass kernels up to n = 64, two at n = 128; each one sums its own
// partial Gram) to keep more of them in flight.
Layout layout(int64_t m, int64_t n, bool oblique, bool csr = false)
{
    Layout L;
    L.np = padded_n(n);
    L.nwg = pass_grid(m, L.np);
    if (csr) {
        const int f = L.np <= 64 ? 4 : (L.np == 128 ? 2 : 1);
        const int64_t panels = (m + 15) / 16;
        int64_t g = (int64_t)L.nwg * f;
        if (g > panels) g = panels;
        if (g > L.nwg) L.nwg = (int)g;
    }
    L.nlvl2 = (L.nwg + 31) / 32;
    L.elems = pass_partial_elems(L.np, oblique);
    const size_t np = (size_t)L.np;
    size_t o = 0;
    L.off_ctl = o;
    o += align256(sizeof(Ctl));
    L.off_G = o;
    o += align256(sizeof(double) * np * (np + 1));
    L.off_Ge = o;
    o += align256(sizeof(double) * np * (np + 1));
    L.off_Rt = o;
    o += align256(sizeof(double) * np * np * SCQR_MAX_PASSES);
    L.off_dinv = o;
    o += align256(sizeof(double) * np * SCQR_MAX_PASSES);
    L.off_R0 = o;
    o += align256(sizeof(double) * np * np);
    L.off_R1 = o;
    o += align256(sizeof(double) * np * np);
    L.off_part = o;
    o += align256(sizeof(double) * (size_t)L.nwg * (size_t)L.elems);
    L.off_lvl2 = o;
    o += align256(sizeof(double) * (size_t)L.nlvl2 * (size_t)L.elems);
    L.off_gsum = o;
    o += align256(sizeof(double) * (size_t)L.elems);
    L.off_bmax = o;
    o += align256(sizeof(double) * (size_t)L.nwg);
    L.off_vprev = o;
    o += align256(sizeof(double) * np);
    L.off_split = o;
    if (L.np == 256) o += align256(sizeof(double) * (2 * 128 * 128 + 2 * 128));
    L.total = o;
    return L;
}

Work carve(void *ws, const Layout &L)
{
    char *c = static_cast<char *>(ws);
    Work w;
    w.ctl = reinterpret_cast<Ctl *>(c + L.off_ctl);
    w.G = reinterpret_cast<double *>(c + L.off_G);
    w.Ge = reinterpret_cast<double *>(c + L.off_Ge);
    w.Rhist = reinterpret_cast<double *>(c + L.off_Rt);
    w.dhist = reinterpret_cast<double *>(c + L.off_dinv);
    w.Racc[0] = reinterpret_cast<double *>(c + L.off_R0);
    w.Racc[1] = reinterpret_cast<double *>(c + L.off_R1);
    w.partials = reinterpret_cast<double *>(c + L.off_part);
    w.lvl2 = reinterpret_cast<double *>(c + L.off_lvl2);
    w.gsum = reinterpret_cast<double *>(c + L.off_gsum);
    w.bmax = reinterpret_cast<double *>(c + L.off_bmax);
    w.vprev = reinterpret_cast<double *>(c + L.off_vprev);
    w.Rsplit = L.np == 256 ? reinterpret_cast<double *>(c + L.off_split) : nullptr;
    w.nwg = L.nwg;
    w.nlvl2 = L.nlvl2;
    w.parts_elems = L.elems;
    return w;
}

bool is_oblique(const scqr_spd_op *B) { return B && (B->kind == SCQR_B_TRIDIAG || B->kind == SCQR_B_CSR); }
bool is_csr(const scqr_spd_op *B) { return B && B->kind == SCQR_B_CSR; }

scqr_status check_B(const scqr_spd_op *B, int64_t m)
{
    if (!B || B->kind == SCQR_B_NONE) return SCQR_OK;
    if (B->kind == SCQR_B_TRIDIAG) {
        if (!B->diag || (m > 1 && !B->off)) return SCQR_E_INVALID;
        return SCQR_OK;
    }
    if (B->kind != SCQR_B_CSR) return SCQR_E_INVALID;
    if (!B->row_ptr || B->nnz < 0 || (B->nnz > 0 && (!B->col || !B->val))) return SCQR_E_INVALID;
    if (m > (int64_t)INT32_MAX) return SCQR_E_UNSUPPORTED;  // 32-bit column indices
    return SCQR_OK;
}

// The operator B of the oblique Gram kernels (tridiagonal or CSR); index errors of a CSR B
// are flagged in the control block.
void set_b(Problem &p, const scqr_spd_op *B, Ctl *ctl)
{
    if (!is_oblique(B)) return;
    if (B->kind == SCQR_B_TRIDIAG) {
        p.bdiag = B->diag;
        p.boff = B->off;
        return;
    }
    p.brp = B->row_ptr;
    p.bcol = B->col;
    p.bval = B->val;
    p.bnnz = B->nnz;
    p.bad_b = &ctl->bad_b;
}

scqr_status hip_status(hipError_t e) { return e == hipSuccess ? SCQR_OK : SCQR_E_HIP; }

// ---------------------------------------------------------------- batched planning
// Instances are grouped by padded width; every class is one launch per step.  A class's rows
// are cut into tasks of at most rpt rows (a multiple of kBatchRowAlign; by default at least
// kBatchMinRows, about kBatchTargetTasks tasks per class, or the caller's tuning); each instance
// is split into ceil(m / rpt) tasks of equal size (up to the alignment), and an instance's tasks
// are contiguous.  The plan depends only on (m_i, n_i), the options and the tuning.
constexpr int kNumClasses = 5;
constexpr int kClassNp[kNumClasses] = {16, 32, 64, 128, 256};
constexpr int64_t kBatchTargetTasks = 4096;
constexpr int64_t kBatchMinRows = 1024;

int class_of(int64_t n)
{
    const int np = padded_n(n);
    for (int c = 0; c < kNumClasses; ++c)
        if (kClassNp[c] == np) return c;
    return -1;
}

struct BatchPlan {
    int P = 0, slots = 0;
    std::vector<int> order;           // instance indices, class-major, ascending within a class
    int cls_first[kNumClasses + 1] = {};
    std::vector<int32_t> ntask;       // per instance
    std::vector<int64_t> task_rows;   // per instance: rows per task (the last one may be shorter)
    int64_t rows_per_task[kNumClasses] = {};
    int panel_rows[kNumClasses] = {};
    int task_first[kNumClasses + 1] = {};
    std::vector<size_t> inst_off;     // per instance: offset of its block in the workspace
    size_t off_inst = 0, off_task = 0, off_blocks = 0, off_part[kNumClasses] = {}, total = 0;
};

size_t inst_block_bytes(int np, int slots)
{
    size_t b = align256(sizeof(Ctl));
    b += align256(sizeof(double) * np * np * slots);
    b += align256(sizeof(double) * np * slots);
    b += align256(sizeof(double) * (size_t)pass_partial_elems(np, false));
    b += align256(sizeof(double) * np);
    if (np > 128) b += align256(sizeof(double) * np * (np + 1)) + 2 * align256(sizeof(double) * np * np);
    return b;
}

scqr_status check_tuning(const scqr_batched_tuning *t)
{
    if (!t) return SCQR_OK;
    for (int c = 0; c < kNumClasses; ++c) {
        if (t->rows_per_task[c] < 0 || t->rows_per_task[c] > ((int64_t)1 << 40)) return SCQR_E_INVALID;
        if (t->panel_rows[c] != 0 && t->panel_rows[c] != 32 && t->panel_rows[c] != 64) return SCQR_E_INVALID;
        if (t->panel_rows[c] == 64 && kClassNp[c] > 64) return SCQR_E_INVALID;
    }
    return SCQR_OK;
}

scqr_status plan_batch(int32_t batch, const int64_t *m, const int64_t *n, const scqr_opts &o,
                       const scqr_batched_tuning *tune, BatchPlan &bp)
{
    scqr_status st = check_opts(&o);
    if (st != SCQR_OK) return st;
    if (o.recompute) return SCQR_E_UNSUPPORTED;
    st = check_tuning(tune);
    if (st != SCQR_OK) return st;
    for (int32_t i = 0; i < batch; ++i) {
        if (n[i] < 1 || m[i] < n[i]) return SCQR_E_INVALID;
        if (n[i] > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    }
    bp.P = o.schedule == SCQR_SCHED_FIXED3 ? 3 : o.schedule == SCQR_SCHED_CHOLQR2 ? 2 : o.max_passes;
    bp.slots = bp.P;
    bp.ntask.assign(batch, 0);
    bp.task_rows.assign(batch, 0);
    bp.inst_off.assign(batch, 0);
    int64_t ntasks = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        bp.cls_first[c] = (int)bp.order.size();
        bp.task_first[c] = (int)ntasks;
        int64_t rows = 0;
        for (int32_t i = 0; i < batch; ++i)
            if (class_of(n[i]) == c) {
                bp.order.push_back(i);
                rows += m[i];
            }
        int64_t rpt;
        if (tune && tune->rows_per_task[c] > 0) {
            rpt = tune->rows_per_task[c];
        } else {
            rpt = (rows + kBatchTargetTasks - 1) / kBatchTargetTasks;
            if (rpt < kBatchMinRows) rpt = kBatchMinRows;
        }
        rpt = (rpt + kBatchRowAlign - 1) / kBatchRowAlign * kBatchRowAlign;
        bp.rows_per_task[c] = rpt;
        bp.panel_rows[c] = (tune && tune->panel_rows[c] == 64) ? 64 : 32;
        for (int k = bp.cls_first[c]; k < (int)bp.order.size(); ++k) {
            const int i = bp.order[k];
            // ceil(m / rpt) tasks of equal size (to a multiple of kBatchRowAlign), not full tasks
            // and a remainder: the longest task of a launch sets its tail
            const int64_t nt = (m[i] + rpt - 1) / rpt;
            int64_t rows_i = (m[i] + nt - 1) / nt;
            rows_i = (rows_i + kBatchRowAlign - 1) / kBatchRowAlign * kBatchRowAlign;
            bp.ntask[i] = (int32_t)((m[i] + rows_i - 1) / rows_i);
            bp.task_rows[i] = rows_i;
            ntasks += bp.ntask[i];
        }
        if (ntasks > INT32_MAX / 2) return SCQR_E_UNSUPPORTED;  // one workgroup per task
    }
    bp.cls_first[kNumClasses] = (int)bp.order.size();
    bp.task_first[kNumClasses] = (int)ntasks;
    size_t o2 = 0;
    bp.off_inst = o2;
    o2 += align256(sizeof(BatchInst) * (size_t)batch);
    bp.off_task = o2;
    o2 += align256(sizeof(BatchTask) * (size_t)ntasks);
    bp.off_blocks = o2;
    for (int32_t i = 0; i < batch; ++i) {
        bp.inst_off[i] = o2;
        o2 += inst_block_bytes(padded_n(n[i]), bp.slots);
    }
    for (int c = 0; c < kNumClasses; ++c) {
        bp.off_part[c] = o2;
        o2 += align256(sizeof(double) * (size_t)(bp.task_first[c + 1] - bp.task_first[c]) *
                       (size_t)pass_partial_elems(kClassNp[c], false));
    }
    bp.total = o2;
    return SCQR_OK;
}

// Arguments of one batched factorization (host arrays of the caller).
struct BatchArgs {
    int32_t batch;
    const int64_t *m, *n;
    const double *const *X;
    const int64_t *ldx;
    double *const *Q;
    const int64_t *ldq;
    double *const *R;
    const int64_t *ldr;
    void *ws;
    size_t ws_bytes;
    scqr_info *infos;
};

int64_t ld_of(const int64_t *ld, int32_t i, const int64_t *n) { return ld ? ld[i] : n[i]; }

// Pointer, leading-dimension, aliasing and workspace checks of a planned batch.
scqr_status check_batch_args(const BatchArgs &a, const BatchPlan &bp)
{
    if (!a.X || !a.Q || !a.R || !a.infos || !a.ws) return SCQR_E_INVALID;
    if (a.ws_bytes < bp.total || (reinterpret_cast<uintptr_t>(a.ws) & 255)) return SCQR_E_WORKSPACE;
    for (int32_t i = 0; i < a.batch; ++i) {
        const int64_t lx = ld_of(a.ldx, i, a.n), lq = ld_of(a.ldq, i, a.n), lr = ld_of(a.ldr, i, a.n);
        if (lx < a.n[i] || lq < a.n[i] || lr < a.n[i]) return SCQR_E_INVALID;
        if (!a.X[i] || !a.Q[i] || !a.R[i]) return SCQR_E_INVALID;
        const size_t xb = mat_bytes(a.m[i], a.n[i], lx), qb = mat_bytes(a.m[i], a.n[i], lq),
                     rb = mat_bytes(a.n[i], a.n[i], lr);
        if (a.Q[i] != a.X[i] && ranges_overlap(a.X[i], xb, a.Q[i], qb)) return SCQR_E_INVALID;
        if (a.Q[i] == a.X[i] && lq != lx) return SCQR_E_INVALID;
        if (ranges_overlap(a.R[i], rb, a.X[i], xb) || ranges_overlap(a.R[i], rb, a.Q[i], qb)) return SCQR_E_INVALID;
        if (ranges_overlap(a.ws, bp.total, a.X[i], xb) || ranges_overlap(a.ws, bp.total, a.Q[i], qb) ||
            ranges_overlap(a.ws, bp.total, a.R[i], rb))
            return SCQR_E_INVALID;
    }
    return SCQR_OK;
}

// The descriptor image (instances in class order, then tasks) for the head of the workspace,
// and the per-class launch descriptions that point into the workspace.
void build_descriptors(const BatchArgs &a, const BatchPlan &bp, std::vector<unsigned char> &host,
                       BatchClass (&cls)[kNumClasses])
{
    char *base = static_cast<char *>(a.ws);
    host.assign(bp.off_blocks, 0);
    BatchInst *hi = reinterpret_cast<BatchInst *>(host.data() + bp.off_inst);
    BatchTask *ht = reinterpret_cast<BatchTask *>(host.data() + bp.off_task);
    const BatchInst *dinst = reinterpret_cast<const BatchInst *>(base + bp.off_inst);
    const BatchTask *dtask = reinterpret_cast<const BatchTask *>(base + bp.off_task);
    for (int c = 0; c < kNumClasses; ++c) {
        const int np = kClassNp[c];
        const int64_t elems = pass_partial_elems(np, false);
        BatchClass &bc = cls[c];
        bc.np = np;
        bc.ninst = bp.cls_first[c + 1] - bp.cls_first[c];
        bc.ntasks = bp.task_first[c + 1] - bp.task_first[c];
        bc.insts = dinst + bp.cls_first[c];
        bc.tasks = dtask + bp.task_first[c];
        bc.partials = reinterpret_cast<double *>(base + bp.off_part[c]);
        bc.vec = true;
        bc.pr = bp.panel_rows[c];
        int t = 0;
        for (int k = bp.cls_first[c]; k < bp.cls_first[c + 1]; ++k) {
            const int i = bp.order[k];
            const int64_t lx = ld_of(a.ldx, i, a.n), lq = ld_of(a.ldq, i, a.n), lr = ld_of(a.ldr, i, a.n);
            BatchInst &I = hi[k];
            I.p.m = a.m[i];
            I.p.n = (int)a.n[i];
            I.p.np = np;
            I.p.X = a.X[i];
            I.p.ldx = lx;
            I.p.Q = a.Q[i];
            I.p.ldq = lq;
            I.p.R = a.R[i];
            I.p.ldr = lr;
            I.p.zero = 0;
            I.p.gram_depth = gram_depth_batched(bp.task_rows[i], bp.ntask[i]);
            char *blk = base + bp.inst_off[i];
            size_t o2 = 0;
            I.w.ctl = reinterpret_cast<Ctl *>(blk + o2);
            o2 += align256(sizeof(Ctl));
            I.w.Rhist = reinterpret_cast<double *>(blk + o2);
            o2 += align256(sizeof(double) * np * np * bp.slots);
            I.w.dhist = reinterpret_cast<double *>(blk + o2);
            o2 += align256(sizeof(double) * np * bp.slots);
            I.w.gsum = reinterpret_cast<double *>(blk + o2);
            o2 += align256(sizeof(double) * elems);
            I.w.vprev = reinterpret_cast<double *>(blk + o2);
            o2 += align256(sizeof(double) * np);
            if (np > 128) {
                I.w.G = reinterpret_cast<double *>(blk + o2);
                o2 += align256(sizeof(double) * np * (np + 1));
                I.w.Racc[0] = reinterpret_cast<double *>(blk + o2);
                o2 += align256(sizeof(double) * np * np);
                I.w.Racc[1] = reinterpret_cast<double *>(blk + o2);
            }
            I.w.parts_elems = elems;
            I.info = a.infos + i;
            I.t0 = t;
            for (int q = 0; q < bp.ntask[i]; ++q, ++t) {
                BatchTask &T = ht[bp.task_first[c] + t];
                T.inst = k - bp.cls_first[c];
                T.r0 = (int64_t)q * bp.task_rows[i];
                const int64_t r1 = T.r0 + bp.task_rows[i];
                T.r1 = r1 < a.m[i] ? r1 : a.m[i];
            }
            I.t1 = t;
            if ((a.n[i] & 1) || (lx & 1) || (lq & 1) || (reinterpret_cast<uintptr_t>(a.X[i]) & 15) ||
                (reinterpret_cast<uintptr_t>(a.Q[i]) & 15) || lx > kBufMaxLd || lq > kBufMaxLd)
                bc.vec = false;
        }
    }
}

SchedParams batch_sched(const scqr_opts &o)
{
    SchedParams sp{};
    sp.schedule = o.schedule;
    sp.shift_mode = o.shift_mode;
    sp.precision = o.precision;
    sp.max_passes = o.max_passes;
    sp.final_gram = 0;
    sp.force_bd = o.debug_force_breakdown_pass;
    sp.zero_shift = o.debug_zero_shift;
    sp.oblique = 0;
    sp.custom_alpha = o.custom_alpha;
    sp.bnorm_user = 0.0;
    sp.trace = nullptr;
    sp.info = nullptr;
    return sp;
}

// The batched schedule: kernels only (no copy, memset or host wait), so that it can be
// captured in a graph once the descriptors are in the workspace.
hipError_t enqueue_batched(hipStream_t s, const BatchPlan &bp, const BatchClass (&cls)[kNumClasses],
                           const scqr_opts &o)
{
    const SchedParams sp = batch_sched(o);
    const bool f32 = o.precision == SCQR_PREC_FP32_FIRST;
    hipError_t e = hipSuccess;
    // one launch per class and step; classes of the same step are independent
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) e = launch_init_b(s, cls[c]);
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
        e = launch_pass_b(s, cls[c], 0, 0, f32, 0);
        if (e == hipSuccess) e = launch_reduce_b(s, cls[c], 0, 0);
        if (e == hipSuccess) e = launch_chol_b(s, cls[c], sp, 1, 0);
    }
    if (f32) {
        for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
            e = launch_pass_b(s, cls[c], 0, -1, false, 0);
            if (e == hipSuccess) e = launch_reduce_b(s, cls[c], -1, 0);
            if (e == hipSuccess) e = launch_chol_b(s, cls[c], sp, 1, 1);
        }
    }
    for (int pass = 1; pass <= bp.P && e == hipSuccess; ++pass) {
        for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
            e = launch_pass_b(s, cls[c], 1, pass, false, 0);
            if (e == hipSuccess) e = launch_reduce_b(s, cls[c], pass, 0);
            if (e == hipSuccess && pass < bp.P) e = launch_chol_b(s, cls[c], sp, pass + 1, 0);
        }
    }
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) e = launch_finalize_b(s, cls[c]);
    return e;
}

// Host-to-device upload of the batched descriptors through pinned staging buffers owned by the
// library (allocated on first use, grown when needed, reused once their last copy completed).
struct Staging {
    void *buf = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
std::mutex g_stage_mu;
Staging g_stage[2];
int g_stage_next = 0;

hipError_t upload(hipStream_t s, void *dst, const void *src, size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging &st = g_stage[g_stage_next];
    g_stage_next ^= 1;
    hipError_t e = hipSuccess;
    if (st.done) {
        e = hipEventSynchronize(st.done);
        if (e != hipSuccess) return e;
    } else {
        e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (st.cap < bytes) {
        if (st.buf) (void)hipHostFree(st.buf);
        st.buf = nullptr;
        st.cap = 0;
        e = hipHostMalloc(&st.buf, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        st.cap = bytes;
    }
    std::memcpy(st.buf, src, bytes);
    e = hipMemcpyAsync(dst, st.buf, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(st.done, s);
}

}  // namespace

// A batched plan: the planned schedule and the descriptor image of one set of buffers, kept in
// the plan's own pinned memory.
struct scqr_batched_plan_s {
    scqr_opts o;
    BatchPlan bp;
    BatchClass cls[kNumClasses];
    std::vector<unsigned char> image;   // descriptor image for the head of ws
    void *ws = nullptr;
    void *pinned = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool uploaded = false;
};

namespace {
}  // namespace

extern "C" {

void scqr_default_opts(scqr_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->schedule = SCQR_SCHED_ADAPTIVE;
    o->shift_mode = SCQR_SHIFT_PAPER;
    o->precision = SCQR_PREC_FP64;
    o->max_passes = 6;
    o->final_gram = 0;
    o->custom_alpha = 0.0;
    o->bnorm = 0.0;
    o->trace = nullptr;
}

const char *scqr_status_string(scqr_status s)
{
    switch (s) {
    case SCQR_OK: return "SCQR_OK";
    case SCQR_E_INVALID: return "SCQR_E_INVALID: invalid argument";
    case SCQR_E_WORKSPACE: return "SCQR_E_WORKSPACE: workspace too small or misaligned";
    case SCQR_E_UNSUPPORTED: return "SCQR_E_UNSUPPORTED: request outside what the library implements";
    case SCQR_E_HIP: return "SCQR_E_HIP: HIP runtime error";
    case SCQR_E_BREAKDOWN: return "SCQR_E_BREAKDOWN: Cholesky factorization broke down";
    case SCQR_E_NOT_CONVERGED: return "SCQR_E_NOT_CONVERGED: max_passes reached";
    case SCQR_E_NONFINITE: return "SCQR_E_NONFINITE: non-finite Gram matrix";
    }
    return "SCQR: unknown status";
}

const char *scqr_build_info(void) { return "scqr 0.1 gfx950 (FP64 MFMA 16x16x4, HIP)"; }

scqr_status scqr_workspace_bytes(int64_t m, int64_t n, const scqr_spd_op *B, const scqr_opts *opts,
                                 size_t *bytes)
{
    if (!bytes || n < 1 || n > SCQR_MAX_N || m < n) return SCQR_E_INVALID;
    if (opts) {
        scqr_status st = check_opts(opts);
        if (st != SCQR_OK) return st;
    }
    *bytes = layout(m, n, is_oblique(B), is_csr(B)).total;
    return SCQR_OK;
}

}  // extern "C"

namespace {

// Validation and enqueue sequence shared by scqr_qr (caller's workspace) and scqr_qr_noalloc
// (the library's static device scratch).
scqr_status qr_enqueue(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                       const scqr_spd_op *B, double *Q, int64_t ldq, double *R, int64_t ldr, void *ws,
                       size_t ws_bytes, const scqr_opts *opts, scqr_info *info)
{
    if (n < 1 || m < n) return SCQR_E_INVALID;
    if (n > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    if (!X || !Q || !R || !ws || !info) return SCQR_E_INVALID;
    if (ldx < n || ldq < n || ldr < n) return SCQR_E_INVALID;
    scqr_opts o;
    if (opts)
        o = *opts;
    else
        scqr_default_opts(&o);
    scqr_status st = check_opts(&o);
    if (st != SCQR_OK) return st;
    st = check_B(B, m);
    if (st != SCQR_OK) return st;
    const bool obl = is_oblique(B);
    if (obl && o.precision == SCQR_PREC_FP32_FIRST) return SCQR_E_UNSUPPORTED;
    if (obl && o.shift_mode == SCQR_SHIFT_DEPTH) return SCQR_E_UNSUPPORTED;
    const bool mt = o.recompute == 1;
    if (mt && (obl || n > 32)) return SCQR_E_UNSUPPORTED;
    // aliasing: Q may equal X exactly; R must not overlap X, Q or the workspace
    const size_t xb = mat_bytes(m, n, ldx), qb = mat_bytes(m, n, ldq), rb = mat_bytes(n, n, ldr);
    if (Q != X && ranges_overlap(X, xb, Q, qb)) return SCQR_E_INVALID;
    if (Q == X && ldq != ldx) return SCQR_E_INVALID;
    if (ranges_overlap(R, rb, X, xb) || ranges_overlap(R, rb, Q, qb)) return SCQR_E_INVALID;
    const Layout L = layout(m, n, obl, is_csr(B));
    if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return SCQR_E_WORKSPACE;
    if (ranges_overlap(ws, L.total, R, rb) || ranges_overlap(ws, L.total, Q, qb) ||
        ranges_overlap(ws, L.total, X, xb))
        return SCQR_E_INVALID;

    hipStream_t s = static_cast<hipStream_t>(stream);
    Work w = carve(ws, L);
    Problem p{};
    p.m = m;
    p.n = (int)n;
    p.np = L.np;
    p.X = X;
    p.ldx = ldx;
    p.Q = Q;
    p.ldq = ldq;
    p.R = R;
    p.ldr = ldr;
    set_b(p, B, w.ctl);
    p.gram_depth = gram_depth_single(m, L.nwg, L.nlvl2);
    SchedParams sp;
    sp.schedule = o.schedule;
    sp.shift_mode = o.shift_mode;
    sp.precision = o.precision;
    sp.max_passes = o.max_passes;
    sp.final_gram = o.final_gram ? 1 : 0;
    sp.force_bd = o.debug_force_breakdown_pass;
    sp.zero_shift = o.debug_zero_shift;
    sp.oblique = obl ? 1 : 0;
    sp.custom_alpha = o.custom_alpha;
    sp.bnorm_user = o.bnorm;
    sp.trace = o.trace;
    sp.info = info;

    const bool f32 = o.precision == SCQR_PREC_FP32_FIRST;
    const int fg = sp.final_gram;
    const int64_t E = pass_partial_elems(L.np, false);
    hipError_t e = launch_init(s, p, w, sp);
    if (e != hipSuccess) return SCQR_E_HIP;
    // pass 1 Gram (binary32 for FP32-first; X^T B X and X^T X for the oblique form)
    e = launch_pass(s, p, w, 0, 0, f32, obl, obl);
    if (e == hipSuccess) e = launch_reduce(s, w, 0, obl ? 2 * E : E, 0);
    if (e == hipSuccess) e = launch_chol(s, p, w, sp, 1, 0);
    if (e == hipSuccess && f32) {
        e = launch_pass(s, p, w, 0, -1, false, false, false);
        if (e == hipSuccess) e = launch_reduce(s, w, -1, E, 0);
        if (e == hipSuccess) e = launch_chol(s, p, w, sp, 1, 1);
    }
    const int P = o.schedule == SCQR_SCHED_FIXED3 ? 3 : o.schedule == SCQR_SCHED_CHOLQR2 ? 2 : o.max_passes;
    for (int pass = 1; pass <= P && e == hipSuccess; ++pass) {
        // stored passes read the previous pass's Q; minimum-traffic passes read X every time
        Problem pp = p;
        if (pass > 1 && !mt) {
            pp.X = Q;
            pp.ldx = ldq;
        }
        e = launch_pass(s, pp, w, (mt ? 5 : 1) | (fg ? 0x100 : 0), pass, false, obl, false);
        if (e == hipSuccess) e = launch_reduce(s, w, pass, E, fg);
        if (e == hipSuccess && pass < P) e = launch_chol(s, p, w, sp, pass + 1, 0);
    }
    if (e == hipSuccess) e = launch_finalize_r(s, p, w, P);
    if (e == hipSuccess && fg) e = launch_final_omega(s, p, w, sp);
    return hip_status(e);
}

// Device scratch of the no-allocation entry point: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is passed to kernels.
constexpr size_t kScratchBytes = (size_t)SCQR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

scqr_status scratch_for_current_device(void **ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SCQR_E_HIP;
    if (dev >= kMaxDevices) return SCQR_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SCQR_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return SCQR_OK;
}

}  // namespace

extern "C" {

scqr_status scqr_qr(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                    const scqr_spd_op *B, double *Q, int64_t ldq, double *R, int64_t ldr, void *ws,
                    size_t ws_bytes, const scqr_opts *opts, scqr_info *info)
{
    return qr_enqueue(stream, m, n, X, ldx, B, Q, ldq, R, ldr, ws, ws_bytes, opts, info);
}

scqr_status scqr_qr_noalloc(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                            const scqr_spd_op *B, double *Q, int64_t ldq, double *R, int64_t ldr,
                            const scqr_opts *opts, scqr_info *info)
{
    // shape and pointer checks first: invalid calls return without any HIP call
    if (n < 1 || m < n) return SCQR_E_INVALID;
    if (n > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    if (!X || !Q || !R || !info) return SCQR_E_INVALID;
    if (ldx < n || ldq < n || ldr < n) return SCQR_E_INVALID;
    scqr_status st = check_B(B, m);
    if (st != SCQR_OK) return st;
    if (opts && (st = check_opts(opts)) != SCQR_OK) return st;
    if (layout(m, n, is_oblique(B), is_csr(B)).total > kScratchBytes) return SCQR_E_WORKSPACE;
    void *ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != SCQR_OK) return st;
    return qr_enqueue(stream, m, n, X, ldx, B, Q, ldq, R, ldr, ws, kScratchBytes, opts, info);
}

scqr_status scqr_gram(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx,
                      const scqr_spd_op *B, double *G, int64_t ldg, void *ws, size_t ws_bytes)
{
    if (n < 1 || m < 1) return SCQR_E_INVALID;
    if (n > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    if (!X || !G || !ws || ldx < n || ldg < n) return SCQR_E_INVALID;
    scqr_status st = check_B(B, m);
    if (st != SCQR_OK) return st;
    const bool obl = is_oblique(B);
    const Layout L = layout(m < n ? n : m, n, obl, is_csr(B));
    if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return SCQR_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Work w = carve(ws, L);
    Problem p{};
    p.m = m;
    p.n = (int)n;
    p.np = L.np;
    p.X = X;
    p.ldx = ldx;
    set_b(p, B, w.ctl);
    const int64_t E = pass_partial_elems(L.np, false);
    SchedParams sp{};
    hipError_t e = launch_init(s, p, w, sp);
    if (e == hipSuccess) e = launch_pass(s, p, w, 0, 0, false, obl, false);
    if (e == hipSuccess) e = launch_reduce(s, w, 0, E, 0);
    if (e == hipSuccess) e = launch_gram_out(s, w, L.np, (int)n, G, ldg);
    return hip_status(e);
}

scqr_status scqr_trsm(void *stream, int64_t m, int64_t n, const double *X, int64_t ldx, const double *R,
                      int64_t ldr, double *Q, int64_t ldq, void *ws, size_t ws_bytes)
{
    if (n < 1 || m < 1) return SCQR_E_INVALID;
    if (n > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    if (!X || !R || !Q || !ws || ldx < n || ldr < n || ldq < n) return SCQR_E_INVALID;
    const size_t xb = mat_bytes(m, n, ldx), qb = mat_bytes(m, n, ldq);
    if (Q != X && ranges_overlap(X, xb, Q, qb)) return SCQR_E_INVALID;
    if (Q == X && ldq != ldx) return SCQR_E_INVALID;
    const Layout L = layout(m < n ? n : m, n, false);
    if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return SCQR_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Work w = carve(ws, L);
    Problem p{};
    p.m = m;
    p.n = (int)n;
    p.np = L.np;
    p.X = X;
    p.ldx = ldx;
    p.Q = Q;
    p.ldq = ldq;
    hipError_t e = launch_set_factor(s, w, L.np, (int)n, R, ldr);
    if (e == hipSuccess) e = launch_pass(s, p, w, 2, 0, false, false, false);
    return hip_status(e);
}

scqr_status scqr_batched_workspace_bytes(int32_t batch, const int64_t *m, const int64_t *n,
                                         const scqr_opts *opts, const scqr_batched_tuning *tune,
                                         size_t *bytes)
{
    if (!bytes || batch < 0 || (batch > 0 && (!m || !n))) return SCQR_E_INVALID;
    scqr_opts o;
    if (opts)
        o = *opts;
    else
        scqr_default_opts(&o);
    BatchPlan bp;
    scqr_status st = plan_batch(batch, m, n, o, tune, bp);
    if (st != SCQR_OK) return st;
    *bytes = bp.total;
    return SCQR_OK;
}

scqr_status scqr_qr_batched(void *stream, int32_t batch, const int64_t *m, const int64_t *n,
                            const double *const *X, const int64_t *ldx, double *const *Q,
                            const int64_t *ldq, double *const *R, const int64_t *ldr, void *ws,
                            size_t ws_bytes, const scqr_opts *opts,
                            const scqr_batched_tuning *tune, scqr_info *infos)
{
    if (batch < 0) return SCQR_E_INVALID;
    if (batch == 0) return SCQR_OK;
    if (!m || !n) return SCQR_E_INVALID;
    scqr_opts o;
    if (opts)
        o = *opts;
    else
        scqr_default_opts(&o);
    if (o.final_gram || o.trace) return SCQR_E_UNSUPPORTED;
    BatchPlan bp;
    scqr_status st = plan_batch(batch, m, n, o, tune, bp);
    if (st != SCQR_OK) return st;
    const BatchArgs a{batch, m, n, X, ldx, Q, ldq, R, ldr, ws, ws_bytes, infos};
    st = check_batch_args(a, bp);
    if (st != SCQR_OK) return st;
    std::vector<unsigned char> host;
    BatchClass cls[kNumClasses];
    build_descriptors(a, bp, host, cls);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = upload(s, ws, host.data(), host.size());
    if (e == hipSuccess) e = enqueue_batched(s, bp, cls, o);
    return hip_status(e);
}

scqr_status scqr_batched_plan_create(int32_t batch, const int64_t *m, const int64_t *n,
                                     const double *const *X, const int64_t *ldx, double *const *Q,
                                     const int64_t *ldq, double *const *R, const int64_t *ldr,
                                     void *ws, size_t ws_bytes, const scqr_opts *opts,
                                     const scqr_batched_tuning *tune, scqr_info *infos,
                                     scqr_batched_plan *plan)
{
    if (!plan) return SCQR_E_INVALID;
    *plan = nullptr;
    if (batch < 1 || !m || !n) return SCQR_E_INVALID;
    scqr_opts o;
    if (opts)
        o = *opts;
    else
        scqr_default_opts(&o);
    if (o.final_gram || o.trace) return SCQR_E_UNSUPPORTED;
    scqr_batched_plan_s *pl = new (std::nothrow) scqr_batched_plan_s();
    if (!pl) return SCQR_E_INVALID;
    pl->o = o;
    scqr_status st = plan_batch(batch, m, n, o, tune, pl->bp);
    const BatchArgs a{batch, m, n, X, ldx, Q, ldq, R, ldr, ws, ws_bytes, infos};
    if (st == SCQR_OK) st = check_batch_args(a, pl->bp);
    if (st != SCQR_OK) {
        delete pl;
        return st;
    }
    build_descriptors(a, pl->bp, pl->image, pl->cls);
    pl->ws = ws;
    pl->bytes = pl->image.size();
    *plan = pl;
    return SCQR_OK;
}

scqr_status scqr_batched_plan_upload(scqr_batched_plan plan, void *stream)
{
    if (!plan) return SCQR_E_INVALID;
    if (!plan->pinned) {
        // the plan's pinned copy of the descriptor image, allocated at the first upload
        if (hipHostMalloc(&plan->pinned, plan->bytes ? plan->bytes : 1, hipHostMallocDefault) != hipSuccess) {
            plan->pinned = nullptr;
            return SCQR_E_HIP;
        }
        if (hipEventCreateWithFlags(&plan->done, hipEventDisableTiming) != hipSuccess) {
            plan->done = nullptr;
            return SCQR_E_HIP;
        }
        std::memcpy(plan->pinned, plan->image.data(), plan->bytes);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(plan->ws, plan->pinned, plan->bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(plan->done, s);
    if (e == hipSuccess) plan->uploaded = true;
    return hip_status(e);
}

scqr_status scqr_batched_plan_run(scqr_batched_plan plan, void *stream)
{
    if (!plan) return SCQR_E_INVALID;
    if (!plan->uploaded) return SCQR_E_INVALID;
    return hip_status(enqueue_batched(static_cast<hipStream_t>(stream), plan->bp, plan->cls, plan->o));
}

scqr_status scqr_batched_plan_destroy(scqr_batched_plan plan)
{
    if (!plan) return SCQR_OK;
    scqr_status st = SCQR_OK;
    if (plan->done) {
        if (plan->uploaded && hipEventSynchronize(plan->done) != hipSuccess) st = SCQR_E_HIP;
        (void)hipEventDestroy(plan->done);
    }
    if (plan->pinned) (void)hipHostFree(plan->pinned);
    delete plan;
    return st;
}

scqr_status scqr_batched_plan_tuning(scqr_batched_plan plan, scqr_batched_tuning *tune, int32_t *ntasks)
{
    if (!plan || !tune) return SCQR_E_INVALID;
    std::memset(tune, 0, sizeof(*tune));
    for (int c = 0; c < kNumClasses; ++c) {
        tune->rows_per_task[c] = plan->bp.rows_per_task[c];
        tune->panel_rows[c] = plan->bp.panel_rows[c];
        if (ntasks) ntasks[c] = plan->bp.task_first[c + 1] - plan->bp.task_first[c];
    }
    return SCQR_OK;
}

scqr_status scqr_backward_workspace_bytes(int64_t m, int64_t n, size_t *bytes)
{
    if (!bytes || n < 1 || n > SCQR_MAX_N || m < n) return SCQR_E_INVALID;
    *bytes = backward_ws_bytes(m, (int)n);
    return SCQR_OK;
}

scqr_status scqr_qr_backward(void *stream, int64_t m, int64_t n, const double *Q, int64_t ldq, const double *R,
                             int64_t ldr, const double *dQ, int64_t lddq, const double *dR, int64_t lddr,
                             double *dX, int64_t lddx, void *ws, size_t ws_bytes)
{
    if (n < 1 || m < n) return SCQR_E_INVALID;
    if (n > SCQR_MAX_N) return SCQR_E_UNSUPPORTED;
    if (!Q || !R || !dX || !ws) return SCQR_E_INVALID;
    if (ldq < n || ldr < n || lddx < n || (dQ && lddq < n) || (dR && lddr < n)) return SCQR_E_INVALID;
    const size_t qb = mat_bytes(m, n, ldq), xb = mat_bytes(m, n, lddx);
    if (ranges_overlap(Q, qb, dX, xb)) return SCQR_E_INVALID;
    if (dQ && dQ != dX && ranges_overlap(dQ, mat_bytes(m, n, lddq), dX, xb)) return SCQR_E_INVALID;
    if (dQ == dX && lddq != lddx) return SCQR_E_INVALID;
    if (ws_bytes < backward_ws_bytes(m, (int)n) || (reinterpret_cast<uintptr_t>(ws) & 255))
        return SCQR_E_WORKSPACE;
    return hip_status(launch_backward(static_cast<hipStream_t>(stream), m, (int)n, Q, ldq, R, ldr, dQ, lddq, dR,
                                      lddr, dX, lddx, ws));
}

scqr_status scqr_profile_enable(int32_t on)
{
    g_prof_on.store(on ? 1 : 0);
    return SCQR_OK;
}

scqr_status scqr_profile_read(scqr_kernel_stat *stats, int32_t capacity, int32_t *count)
{
    if (!count || capacity < 0 || (capacity > 0 && !stats)) return SCQR_E_INVALID;
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    std::vector<scqr_kernel_stat> agg;
    scqr_status st = SCQR_OK;
    for (auto &r : recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            st = SCQR_E_HIP;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        scqr_kernel_stat z;
        std::memset(&z, 0, sizeof(z));
        std::strncpy(z.name, r.name.c_str(), sizeof(z.name) - 1);
        z.launches = 1;
        z.total_ms = ms;
        agg.push_back(z);
    }
    const int32_t nout = (int32_t)agg.size() < capacity ? (int32_t)agg.size() : capacity;
    for (int32_t i = 0; i < nout; ++i) stats[i] = agg[i];
    *count = (int32_t)agg.size();
    return st;
}

}  // extern "C"
