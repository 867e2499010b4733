// Host driver and C ABI: Algorithm I / Algorithm II / FP64-only CG state
// machine, 2BFS driver, workspace planning.  Kernels are enqueued ahead on the
// context stream; the host polls one device-state snapshot per group of
// iterations while the next group is already queued.

#include "mpcg_internal.hpp"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace mpcg;

struct mpcg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    mpcg_options opt{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    DevState *hst = nullptr;   // pinned: [0],[1] poll snapshots, [2] synchronous reads
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t tm[8] = {};
    KnnModel model;
    bool has_model = false;
    float last_kernel_ms = 0.0f;
};

#define HIPCHK(x)                                        \
    do {                                                 \
        if ((x) != hipSuccess) return MPCG_EDEVICE;      \
    } while (0)

namespace mpcg {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout plan_layout(int64_t n, int64_t nnz)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t N = (size_t)n, M = (size_t)(nnz > 0 ? nnz : 1);
    L.n = n;
    L.nnz = nnz;
    L.part_cap = (n + 31) / 32 + 64;   // SpMV blocks hold >= 32 rows; vector blocks 1024
    L.state = take(sizeof(DevState));
    L.part = take(sizeof(double) * 2 * (size_t)L.part_cap);
    L.rp32 = take(sizeof(int32_t) * (N + 1));
    L.val32 = take(sizeof(float) * M);
    L.x32 = take(sizeof(float) * N);
    L.r32 = take(sizeof(float) * N);
    L.q32 = take(sizeof(float) * N);
    L.dA32 = take(sizeof(float) * N);
    L.dB32 = take(sizeof(float) * N);
    L.r64 = take(sizeof(double) * N);
    L.q64 = take(sizeof(double) * N);
    L.dA64 = take(sizeof(double) * N);
    L.dB64 = take(sizeof(double) * N);
    L.dist = take(sizeof(int32_t) * N);
    L.q0 = take(sizeof(int32_t) * N);
    L.q1 = take(sizeof(int32_t) * N);
    L.label = take(sizeof(int32_t) * N);
    L.tarr = take(sizeof(int32_t) * N);
    L.best = take(sizeof(unsigned long long) * N);
    L.total = off;
    return L;
}

int spmv_rows_per_block(int64_t n, int64_t nnz, int value_bytes)
{
    const int64_t chunk = kLdsBytes / (2 * value_bytes);
    int64_t avg = n > 0 ? (nnz + n - 1) / n : 1;
    if (avg < 1) avg = 1;
    int64_t R = chunk / avg;
    R = (R / 32) * 32;
    if (R < 32) R = 32;
    if (R > kBlock) R = kBlock;
    return (int)R;
}

}  // namespace mpcg

namespace {

struct Plan {
    Layout L;
    int32_t n = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
    DevState *st = nullptr;
    double *part = nullptr;
    int R32 = 256, R64 = 256;
    char *ws = nullptr;
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

mpcg_status read_state(mpcg_ctx *c, const Plan &p, DevState *out)
{
    HIPCHK(hipMemcpyAsync(&c->hst[2], p.st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *out = c->hst[2];
    return MPCG_OK;
}

// Validate A (and b) on the device, convert row pointers / cast values when
// asked, and read back the verdict before any result buffer is touched.
mpcg_status ingest(mpcg_ctx *c, const mpcg_csr *A, const double *b, bool need_val32, Plan *p)
{
    if (!c || !A || A->n <= 0 || A->n >= 0x7fffffff || A->nnz < 0 || A->nnz >= 0x7fffffff ||
        !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return MPCG_EINVAL;
    p->L = plan_layout(A->n, A->nnz);
    if (!c->ws || c->ws_bytes < p->L.total) return MPCG_ENOMEM;
    p->ws = c->ws;
    p->n = (int32_t)A->n;
    p->nnz = A->nnz;
    p->col = A->col_idx;
    p->val = A->val;
    p->st = p->at<DevState>(p->L.state);
    p->part = p->at<double>(p->L.part);
    int32_t *rp32 = A->row_ptr_is_i64 ? p->at<int32_t>(p->L.rp32) : nullptr;
    p->rp = A->row_ptr_is_i64 ? rp32 : static_cast<const int32_t *>(A->row_ptr);
    HIPCHK(hipMemsetAsync(p->st, 0, sizeof(DevState), c->stream));
    launch_ingest(c->stream, A->row_ptr, A->row_ptr_is_i64 ? 1 : 0, A->col_idx, A->val, b, p->n,
                  A->nnz, rp32, need_val32 ? p->at<float>(p->L.val32) : nullptr, p->st);
    HIPCHK(hipGetLastError());
    DevState s;
    mpcg_status rc = read_state(c, *p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.ing_err & (kErrRowPtr | kErrCol | kErrUnsorted)) return MPCG_EINVAL;
    if (s.ing_err & (kErrNonFiniteA | kErrNonFiniteB)) return MPCG_ENONFINITE;
    p->R64 = spmv_rows_per_block(A->n, A->nnz, 8);
    p->R32 = spmv_rows_per_block(A->n, A->nnz, 4);
    return MPCG_OK;
}

int poll_iters(const mpcg_ctx *c) { return c->opt.graph_iters > 0 ? c->opt.graph_iters : 8; }

// Run CG iterations in precision T until the device says stop.  Groups of
// iterations are enqueued one ahead of the state snapshot being inspected.
template <typename T>
mpcg_status cg_loop(mpcg_ctx *c, const Plan &p, const T *val, int R, T *x, T *r, T *q, T *dA,
                    T *dB, DevState *out)
{
    const int G = poll_iters(c);
    int64_t k = 0;
    for (;;) {
        for (int g = 0; g < G; ++g) {
            launch_cg_spmv<T>(c->stream, p.rp, p.col, val, p.n, R, r, dA, dB, q, p.part, p.st);
            launch_cg_update<T>(c->stream, p.n, x, r, q, dA, dB, p.part, p.st);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&c->hst[k & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipEventRecord(c->ev[k & 1], c->stream));
        if (k > 0) {
            HIPCHK(hipEventSynchronize(c->ev[(k - 1) & 1]));
            if (!c->hst[(k - 1) & 1].live) break;
        }
        ++k;
    }
    return read_state(c, p, out);
}

BfsBufs bfs_bufs(const Plan &p)
{
    BfsBufs b{};
    b.rp = p.rp;
    b.col = p.col;
    b.n = p.n;
    const int64_t avg = (p.nnz + p.n - 1) / p.n;
    int lanes = 1;
    while (lanes < avg && lanes < 32) lanes <<= 1;
    b.lanes = lanes;
    b.dist = p.at<int32_t>(p.L.dist);
    b.q0 = p.at<int32_t>(p.L.q0);
    b.q1 = p.at<int32_t>(p.L.q1);
    b.label = p.at<int32_t>(p.L.label);
    b.tarr = p.at<int32_t>(p.L.tarr);
    b.best = p.at<unsigned long long>(p.L.best);
    b.st = p.st;
    return b;
}

mpcg_status bfs_run(mpcg_ctx *c, const Plan &p, const BfsBufs &bb, DevState *out)
{
    const int levels = 16;
    for (int64_t round = 0;; ++round) {
        launch_bfs_round(c->stream, bb, levels);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&c->hst[round & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipEventRecord(c->ev[round & 1], c->stream));
        if (round > 0) {
            HIPCHK(hipEventSynchronize(c->ev[(round - 1) & 1]));
            if (c->hst[(round - 1) & 1].bfs_done) break;
        }
        if (round > (int64_t)p.n + 4) return MPCG_EDEVICE;   // every round expands >= 1 level
    }
    return read_state(c, p, out);
}

// 2BFS per component; fills pdiam, bfs_t, bfs_u, n_components.
mpcg_status pseudo_diameter(mpcg_ctx *c, const Plan &p, mpcg_features_t *f)
{
    BfsBufs bb = bfs_bufs(p);
    DevState s;
    launch_bfs_seed_single(c->stream, bb, 0);
    mpcg_status rc = bfs_run(c, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    if (s.bfs_visited == p.n) {
        const int32_t t = s.bfs_far;
        launch_bfs_seed_single(c->stream, bb, t);
        rc = bfs_run(c, p, bb, &s);
        if (rc != MPCG_OK) return rc;
        f->pdiam = s.bfs_level;
        f->bfs_t = t;
        f->bfs_u = s.bfs_far;
        f->n_components = 1;
        return MPCG_OK;
    }
    launch_cc(c->stream, bb);
    launch_bfs_seed_roots(c->stream, bb);
    rc = bfs_run(c, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    launch_comp_argmax(c->stream, bb, 0);
    launch_bfs_seed_far(c->stream, bb);
    rc = bfs_run(c, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    launch_comp_argmax(c->stream, bb, 1);
    launch_comp_final(c->stream, bb);
    HIPCHK(hipGetLastError());
    rc = read_state(c, p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.guard) return MPCG_EDEVICE;
    const uint64_t key = s.comp_best;
    const int32_t comp = (int32_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
    int32_t t = 0;
    unsigned long long bu = 0;
    HIPCHK(hipMemcpyAsync(&t, bb.tarr + comp, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&bu, bb.best + comp, sizeof(bu), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    f->pdiam = (int64_t)(key >> 32);
    f->bfs_t = t;
    f->bfs_u = (int64_t)(0xffffffffu - (uint32_t)(bu & 0xffffffffull));
    f->n_components = s.ncomp;
    return MPCG_OK;
}

// FP32 prefix of Algorithm II: k0 iterations without the eps1 test.
mpcg_status fp32_prefix(mpcg_ctx *c, const Plan &p, const double *b, int32_t k0, DevState *s)
{
    float *x = p.at<float>(p.L.x32), *r = p.at<float>(p.L.r32), *q = p.at<float>(p.L.q32);
    float *dA = p.at<float>(p.L.dA32), *dB = p.at<float>(p.L.dB32);
    // thr = 0: only gamma' = 0 or a breakdown ends the prefix before k0
    launch_init32(c->stream, b, x, r, dA, p.n, 0.0, 1, k0, k0, p.part, p.st);
    HIPCHK(hipGetLastError());
    mpcg_status rc = read_state(c, p, s);
    if (rc != MPCG_OK) return rc;
    if (s->live) rc = cg_loop<float>(c, p, p.at<float>(p.L.val32), p.R32, x, r, q, dA, dB, s);
    return rc;
}

double v_from_ratios(const DevState &s, int32_t used)
{
    double sum = 0.0;
    for (int i = 0; i < used; ++i) sum = sum + s.ratios[i];
    return used > 0 ? sum / (double)used : 0.0;
}

const double kEpsClass[8] = {0, 0, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7};

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0f;
    return ms;
}

}  // namespace

extern "C" {

const char *mpcg_strerror(mpcg_status s)
{
    switch (s) {
    case MPCG_OK: return "ok";
    case MPCG_EINVAL: return "invalid argument or malformed CSR";
    case MPCG_ENOTSPD: return "matrix not positive definite (d^T A d <= 0)";
    case MPCG_ENOCONV: return "no convergence within the iteration or restart cap";
    case MPCG_ENOMEM: return "workspace missing or too small";
    case MPCG_EDEVICE: return "HIP runtime error or device guard";
    case MPCG_ENONFINITE: return "non-finite value";
    case MPCG_EBUSY: return "busy";
    case MPCG_ECANCELED: return "cancelled";
    case MPCG_ENOMODEL: return "no kNN model loaded";
    }
    return "unknown status";
}

mpcg_status mpcg_create(mpcg_ctx **out, const mpcg_options *opt, void *hip_stream)
{
    if (!out) return MPCG_EINVAL;
    *out = nullptr;
    mpcg_options o{};
    o.k0 = 20;
    o.max_restarts = 5;
    if (opt) {
        o = *opt;
        if (o.k0 <= 0) o.k0 = 20;
        if (o.max_restarts < 0) return MPCG_EINVAL;
    }
    if (o.k0 > kK0Max || o.tol_mode < 0 || o.tol_mode > 1 || o.knn_k < 0 || o.graph_iters < 0)
        return MPCG_EINVAL;
    mpcg_ctx *c = new (std::nothrow) mpcg_ctx();
    if (!c) return MPCG_EDEVICE;
    c->opt = o;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipHostMalloc((void **)&c->hst, 3 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MPCG_EDEVICE;
    }
    for (auto &e : c->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MPCG_EDEVICE;
    for (auto &e : c->tm)
        if (hipEventCreate(&e) != hipSuccess) return MPCG_EDEVICE;
    *out = c;
    return MPCG_OK;
}

mpcg_status mpcg_destroy(mpcg_ctx *c)
{
    if (!c) return MPCG_EINVAL;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->tm) if (e) (void)hipEventDestroy(e);
    if (c->hst) (void)hipHostFree(c->hst);
    knn_free(&c->model);
    delete c;
    return MPCG_OK;
}

mpcg_status mpcg_workspace_size(const mpcg_ctx *c, int64_t n, int64_t nnz, size_t *bytes)
{
    if (!c || !bytes || n <= 0 || nnz < 0) return MPCG_EINVAL;
    *bytes = plan_layout(n, nnz).total;
    return MPCG_OK;
}

mpcg_status mpcg_set_workspace(mpcg_ctx *c, void *arena, size_t bytes)
{
    if (!c || (arena == nullptr && bytes > 0) || ((uintptr_t)arena & 255) != 0) return MPCG_EINVAL;
    c->ws = static_cast<char *>(arena);
    c->ws_bytes = bytes;
    return MPCG_OK;
}

mpcg_status mpcg_load_model(mpcg_ctx *c, const char *path)
{
    if (!c || !path) return MPCG_EINVAL;
    KnnModel m;
    if (knn_load(path, &m) != 0) return MPCG_EINVAL;
    knn_free(&c->model);
    c->model = m;
    c->has_model = true;
    return MPCG_OK;
}

mpcg_status mpcg_select_eps1(const mpcg_ctx *c, const mpcg_features_t *f, double *eps1, int32_t *cls)
{
    if (!c || !f) return MPCG_EINVAL;
    if (!c->has_model || c->model.ns <= 0) return MPCG_ENOMODEL;
    const double chi[4] = {(double)f->n, (double)f->m, (double)f->pdiam, f->v};
    int32_t exact = 0;
    const int t = knn_select(c->model, chi, c->opt.knn_k, &exact);
    if (t < 2 || t > 7) return MPCG_EINVAL;
    if (eps1) *eps1 = kEpsClass[t];
    if (cls) *cls = t;
    return MPCG_OK;
}

mpcg_status mpcg_features(mpcg_ctx *c, const mpcg_csr *A, const double *b, int32_t k0,
                          mpcg_features_t *out)
{
    if (!c || !b || !out || k0 <= 0 || k0 > kK0Max) return MPCG_EINVAL;
    Plan p;
    mpcg_status rc = ingest(c, A, b, true, &p);
    if (rc != MPCG_OK) return rc;
    mpcg_features_t f{};
    f.n = A->n;
    f.m = A->nnz;
    rc = pseudo_diameter(c, p, &f);
    if (rc != MPCG_OK) return rc;
    DevState s;
    rc = fp32_prefix(c, p, b, k0, &s);
    if (rc != MPCG_OK) return rc;
    f.k0_used = s.iter;
    f.v = v_from_ratios(s, s.iter);
    *out = f;
    return MPCG_OK;
}

mpcg_status mpcg_solve(mpcg_ctx *c, const mpcg_csr *A, const double *b, double *x, double eps1,
                       double eps2, mpcg_stats *stats)
{
    if (!c || !A || !b || !x) return MPCG_EINVAL;
    if (!(eps2 > 0.0) || !std::isfinite(eps2)) return MPCG_EINVAL;
    const bool autoe = (eps1 == MPCG_EPS1_AUTO);
    const bool dponly = (eps1 == MPCG_EPS1_NONE);
    if (!autoe && !dponly && !(eps1 > 0.0 && std::isfinite(eps1))) return MPCG_EINVAL;
    if (autoe && (!c->has_model || c->model.ns <= 0)) return MPCG_ENOMODEL;

    mpcg_stats S{};
    S.eps1_class = -1;
    S.eps1_used = dponly ? -1.0 : eps1;
    HIPCHK(hipEventRecord(c->tm[0], c->stream));
    Plan p;
    mpcg_status rc = ingest(c, A, b, !dponly, &p);
    if (rc != MPCG_OK) { S.status = rc; if (stats) *stats = S; return rc; }
    const int abs_tol = c->opt.tol_mode == 1;
    const int64_t n = A->n;
    int64_t mi1 = c->opt.maxit1 > 0 ? c->opt.maxit1 : n;
    int64_t mi2 = c->opt.maxit2 > 0 ? c->opt.maxit2 : (10 * n > 1000 ? 10 * n : 1000);
    const int32_t maxit1 = (int32_t)(mi1 < 0x7ffffff0 ? mi1 : 0x7ffffff0);
    const int32_t maxit2 = (int32_t)(mi2 < 0x7ffffff0 ? mi2 : 0x7ffffff0);

    double *r64 = p.at<double>(p.L.r64), *q64 = p.at<double>(p.L.q64);
    double *dA64 = p.at<double>(p.L.dA64), *dB64 = p.at<double>(p.L.dB64);
    DevState s;
    bool feat_timed = false;
    double bnorm = 0.0;

    if (!dponly) {
        float *x32 = p.at<float>(p.L.x32), *r32 = p.at<float>(p.L.r32), *q32 = p.at<float>(p.L.q32);
        float *dA32 = p.at<float>(p.L.dA32), *dB32 = p.at<float>(p.L.dB32);
        const float *val32 = p.at<float>(p.L.val32);
        bool broke = false;
        if (autoe) {
            HIPCHK(hipEventRecord(c->tm[1], c->stream));
            mpcg_features_t f{};
            f.n = n;
            f.m = A->nnz;
            rc = pseudo_diameter(c, p, &f);
            if (rc != MPCG_OK) { S.status = rc; if (stats) *stats = S; return rc; }
            HIPCHK(hipEventRecord(c->tm[2], c->stream));
            feat_timed = true;
            rc = fp32_prefix(c, p, b, c->opt.k0, &s);
            if (rc != MPCG_OK) { S.status = rc; if (stats) *stats = S; return rc; }
            if (s.bnorm2 == 0.0) goto zero_rhs;
            f.k0_used = s.iter;
            f.v = v_from_ratios(s, s.iter);
            S.feat = f;
            broke = (s.reason == kNotSpd || s.reason == kNonFinite);
            const double chi[4] = {(double)f.n, (double)f.m, (double)f.pdiam, f.v};
            int32_t exact = 0;
            const int cls = knn_select(c->model, chi, c->opt.knn_k, &exact);
            if (cls < 2 || cls > 7) { S.status = MPCG_EINVAL; if (stats) *stats = S; return MPCG_EINVAL; }
            const double e1 = kEpsClass[cls];
            S.eps1_class = cls;
            S.eps1_used = e1;
            if (exact) S.flags |= MPCG_FLAG_KNN_EXACT;
            if (!broke) {
                const double thr1 = abs_tol ? e1 : e1 * std::sqrt(s.bnorm2);
                launch_set_phase(c->stream, p.st, thr1, maxit1, c->opt.k0, 0);
                HIPCHK(hipGetLastError());
                rc = read_state(c, p, &s);
                if (rc != MPCG_OK) return rc;
                if (s.live) rc = cg_loop<float>(c, p, val32, p.R32, x32, r32, q32, dA32, dB32, &s);
                if (rc != MPCG_OK) return rc;
            }
        } else {
            launch_init32(c->stream, b, x32, r32, dA32, p.n, eps1, abs_tol, maxit1, 0, p.part, p.st);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
            if (s.bnorm2 == 0.0) goto zero_rhs;
            if (s.live) rc = cg_loop<float>(c, p, val32, p.R32, x32, r32, q32, dA32, dB32, &s);
            if (rc != MPCG_OK) return rc;
        }
        if (s.reason == kNotSpd || s.reason == kNonFinite) S.flags |= MPCG_FLAG_FP32_BREAKDOWN;
        else if (s.reason == kMaxit) S.flags |= MPCG_FLAG_FP32_MAXIT;
        S.n1 = s.iter;
        bnorm = std::sqrt(s.bnorm2);
        S.relres_sp = std::sqrt(s.gamma) / bnorm;
        HIPCHK(hipEventRecord(c->tm[3], c->stream));
        // restart in FP64 from float64(x~) with a freshly computed residual
        launch_set_phase(c->stream, p.st, 0.0, 0, 0, 1);
        launch_restart(c->stream, p.rp, p.col, p.val, p.n, p.R64, x32, x, b, r64, dA64, dB64, eps2,
                       abs_tol, maxit2, p.part, p.st);
        HIPCHK(hipGetLastError());
    } else {
        // FP64-only CG from x0 = 0 through the restart kernel: r = b - A*0 = b
        // exactly, with the same reductions as the mixed path's restart.
        HIPCHK(hipEventRecord(c->tm[3], c->stream));
        launch_fill_f64(c->stream, x, n, 0.0);
        launch_restart(c->stream, p.rp, p.col, p.val, p.n, p.R64, nullptr, x, b, r64, dA64, dB64, eps2,
                       abs_tol, maxit2, p.part, p.st);
        HIPCHK(hipGetLastError());
    }
    rc = read_state(c, p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.bnorm2 == 0.0) goto zero_rhs;
    bnorm = std::sqrt(s.bnorm2);
    S.relres_restart_true = std::sqrt(s.gamma) / bnorm;
    {
        const double thr2 = abs_tol ? eps2 : eps2 * bnorm;
        for (;;) {
            if (s.live) {
                rc = cg_loop<double>(c, p, p.val, p.R64, x, r64, q64, dA64, dB64, &s);
                if (rc != MPCG_OK) return rc;
            }
            if (s.reason == kMaxit) { rc = MPCG_ENOCONV; break; }
            if (s.reason == kNotSpd) { rc = MPCG_ENOTSPD; break; }
            if (s.reason == kNonFinite) { rc = MPCG_ENONFINITE; break; }
            launch_resid(c->stream, p.rp, p.col, p.val, p.n, p.R64, x, b, p.part, p.st);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
            const double rho = std::sqrt(s.resid2);
            S.relres_final_true = rho / bnorm;
            if (rho <= thr2) { rc = MPCG_OK; break; }
            if (S.restarts >= c->opt.max_restarts) { rc = MPCG_ENOCONV; break; }
            S.restarts++;
            S.flags |= MPCG_FLAG_FINAL_RESTARTED;
            launch_restart(c->stream, p.rp, p.col, p.val, p.n, p.R64, nullptr, x, b, r64, dA64, dB64,
                           eps2, abs_tol, maxit2, p.part, p.st);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
        }
        if (rc != MPCG_OK && S.relres_final_true == 0.0) {
            launch_resid(c->stream, p.rp, p.col, p.val, p.n, p.R64, x, b, p.part, p.st);
            DevState s2;
            if (read_state(c, p, &s2) == MPCG_OK) S.relres_final_true = std::sqrt(s2.resid2) / bnorm;
        }
    }
    S.n2 = s.iter;
    HIPCHK(hipEventRecord(c->tm[4], c->stream));
    HIPCHK(hipEventSynchronize(c->tm[4]));
    S.t_total_ms = elapsed(c->tm[0], c->tm[4]);
    S.t_dp_ms = elapsed(c->tm[3], c->tm[4]);
    S.t_sp_ms = dponly ? 0.0 : elapsed(c->tm[0], c->tm[3]);
    if (feat_timed) {
        S.t_feat_ms = elapsed(c->tm[1], c->tm[2]);
        S.t_sp_ms -= S.t_feat_ms;
    }
    if (S.n1 > 0 && S.n2 > 0 && S.t_dp_ms > 0.0)
        S.omega_measured = (S.t_sp_ms / S.n1) / (S.t_dp_ms / S.n2);
    S.I_third = S.n1 / 3.0 + S.n2;
    S.I_meas = S.omega_measured * S.n1 + S.n2;
    S.status = rc;
    if (stats) *stats = S;
    return rc;

zero_rhs:
    launch_fill_f64(c->stream, x, n, 0.0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    S.n1 = 0;
    S.n2 = 0;
    S.status = MPCG_OK;
    if (stats) *stats = S;
    return MPCG_OK;
}

mpcg_status mpcg_spmv(mpcg_ctx *c, const mpcg_csr *A, int32_t precision, const void *x, void *y)
{
    if (!c || !x || !y || (precision != 32 && precision != 64)) return MPCG_EINVAL;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, precision == 32, &p);
    if (rc != MPCG_OK) return rc;
    HIPCHK(hipEventRecord(c->tm[5], c->stream));
    if (precision == 64)
        launch_spmv_plain<double>(c->stream, p.rp, p.col, p.val, p.n, p.R64,
                                  static_cast<const double *>(x), static_cast<double *>(y));
    else
        launch_spmv_plain<float>(c->stream, p.rp, p.col, p.at<float>(p.L.val32), p.n, p.R32,
                                 static_cast<const float *>(x), static_cast<float *>(y));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->tm[6], c->stream));
    HIPCHK(hipEventSynchronize(c->tm[6]));
    c->last_kernel_ms = elapsed(c->tm[5], c->tm[6]);
    return MPCG_OK;
}

mpcg_status mpcg_bfs(mpcg_ctx *c, const mpcg_csr *A, int64_t src, int32_t *dist, int64_t *ecc,
                     int64_t *far)
{
    if (!c || !A || !dist || src < 0 || src >= A->n) return MPCG_EINVAL;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, false, &p);
    if (rc != MPCG_OK) return rc;
    BfsBufs bb = bfs_bufs(p);
    launch_bfs_seed_single(c->stream, bb, (int32_t)src);
    DevState s;
    rc = bfs_run(c, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    HIPCHK(hipMemcpyAsync(dist, bb.dist, sizeof(int32_t) * (size_t)p.n, hipMemcpyDeviceToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (ecc) *ecc = s.bfs_level;
    if (far) *far = s.bfs_far;
    return MPCG_OK;
}

mpcg_status mpcg_last_kernel_ms(const mpcg_ctx *c, double *ms)
{
    if (!c || !ms) return MPCG_EINVAL;
    *ms = c->last_kernel_ms;
    return MPCG_OK;
}

mpcg_status mpcg_time_kernel(mpcg_ctx *c, const mpcg_csr *A, int32_t kernel, int32_t reps, double *ms)
{
    if (!c || !A || !ms || reps < 1 || kernel < 0 || kernel > 5) return MPCG_EINVAL;
    const bool f32 = (kernel & 1) != 0;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, f32, &p);
    if (rc != MPCG_OK) return rc;
    float *x32 = p.at<float>(p.L.x32), *r32 = p.at<float>(p.L.r32), *q32 = p.at<float>(p.L.q32);
    float *dA32 = p.at<float>(p.L.dA32), *dB32 = p.at<float>(p.L.dB32);
    double *r64 = p.at<double>(p.L.r64), *q64 = p.at<double>(p.L.q64);
    double *dA64 = p.at<double>(p.L.dA64), *dB64 = p.at<double>(p.L.dB64);
    double *x64 = p.at<double>(p.L.best);   // the BFS key array doubles as x here
    if (f32) {
        launch_fill_f32(c->stream, x32, p.n, 0.0f);
        launch_fill_f32(c->stream, r32, p.n, 1.0f);
        launch_fill_f32(c->stream, q32, p.n, 0.5f);
        launch_fill_f32(c->stream, dA32, p.n, 0.25f);
        launch_fill_f32(c->stream, dB32, p.n, 0.25f);
    } else {
        launch_fill_f64(c->stream, x64, p.n, 0.0);
        launch_fill_f64(c->stream, r64, p.n, 1.0);
        launch_fill_f64(c->stream, q64, p.n, 0.5);
        launch_fill_f64(c->stream, dA64, p.n, 0.25);
        launch_fill_f64(c->stream, dB64, p.n, 0.25);
    }
    launch_timing_state(c->stream, p.st);
    HIPCHK(hipGetLastError());
    auto one = [&]() {
        switch (kernel) {
        case MPCG_KERNEL_CG_SPMV_F64:
            launch_cg_spmv<double>(c->stream, p.rp, p.col, p.val, p.n, p.R64, r64, dA64, dB64, q64, p.part, p.st);
            break;
        case MPCG_KERNEL_CG_SPMV_F32:
            launch_cg_spmv<float>(c->stream, p.rp, p.col, p.at<float>(p.L.val32), p.n, p.R32, r32, dA32, dB32,
                                  q32, p.part, p.st);
            break;
        case MPCG_KERNEL_UPDATE_F64:
            launch_cg_update<double>(c->stream, p.n, x64, r64, q64, dA64, dB64, p.part, p.st);
            break;
        case MPCG_KERNEL_UPDATE_F32:
            launch_cg_update<float>(c->stream, p.n, x32, r32, q32, dA32, dB32, p.part, p.st);
            break;
        case MPCG_KERNEL_SPMV_F64:
            launch_spmv_plain<double>(c->stream, p.rp, p.col, p.val, p.n, p.R64, r64, q64);
            break;
        default:
            launch_spmv_plain<float>(c->stream, p.rp, p.col, p.at<float>(p.L.val32), p.n, p.R32, r32, q32);
            break;
        }
    };
    one();   // warm caches and code
    HIPCHK(hipEventRecord(c->tm[5], c->stream));
    for (int i = 0; i < reps; ++i) one();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->tm[6], c->stream));
    HIPCHK(hipEventSynchronize(c->tm[6]));
    DevState s;
    rc = read_state(c, p, &s);
    if (rc != MPCG_OK) return rc;
    if (!s.live) return MPCG_EDEVICE;   // a launch exited early: the timing would be wrong
    *ms = elapsed(c->tm[5], c->tm[6]) / reps;
    return MPCG_OK;
}

}  // extern "C"
