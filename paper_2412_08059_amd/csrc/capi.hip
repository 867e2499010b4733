// Host driver and C ABI: Algorithm I / Algorithm II / FP64-only CG state
// machine, 2BFS driver, workspace planning.  Kernels are enqueued ahead on the
// context stream; the host polls one device-state snapshot per group of
// iterations while the next group is already queued.

#include "batch_internal.hpp"
#include "mpcg_internal.hpp"
#include "tune.hpp"

#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace mpcg;

// ---- workspace of mpcg_solve_noalloc: one array per GPU, in the code object.
// In host code `scratch` only names the symbol; its device address on each GPU
// comes from hipGetSymbolAddress at context creation (with that device
// current) and is the only form host code passes on.
constexpr size_t kNoAllocBytes = (size_t)160 << 20;   // 160 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Called by mpcg_create with the context's device current; once per device.
hipError_t scratch_init(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) g_scratch_ptr[dev] = ptr;
    return e == hipSuccess && !ptr ? hipErrorInvalidSymbol : e;
}

void *scratch_of(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
}
}  // namespace

// A stream plus the pinned snapshots and events used to poll the device state
// from it.
// A round of bit-parallel level launches captured as a graph, replayed while
// its arguments stay the same.
struct DiaGraph {
    hipStream_t cap = nullptr;   // capture stream (owned)
    hipGraphExec_t exec = nullptr;
    BfsBufs key{};               // the arguments it was captured with
    bool failed = false;         // capture unavailable: plain launches
    bool suspended = false;      // plain launches (mpcg_solve_noalloc: the graph runtime allocates)
};

struct Chan {
    hipStream_t s = nullptr;
    DevState *poll[2] = {nullptr, nullptr};
    DevState *sync = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    DiaGraph *dia = nullptr;     // owned
};

bool same_dia_args(const BfsBufs &a, const BfsBufs &b)
{
    return a.df0 == b.df0 && a.df1 == b.df1 && a.dv == b.dv && a.dm == b.dm && a.dist == b.dist && a.st == b.st &&
           a.part_cnt == b.part_cnt && a.part_min == b.part_min && a.dia_two == b.dia_two &&
           a.nwords == b.nwords && a.dia_grid == b.dia_grid && std::memcmp(&a.doff, &b.doff, sizeof(DiaOffs)) == 0;
}

// One round: a replay of the captured graph (captured again when the
// arguments change), else plain launches.
void dia_round(const Chan &ch, const BfsBufs &bb)
{
    DiaGraph *g = ch.dia;
    if (g && !g->failed && !g->suspended) {
        if (!g->exec || !same_dia_args(g->key, bb)) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            g->exec = nullptr;
            hipGraph_t gr = nullptr;
            bool ok = (g->cap || hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) == hipSuccess) &&
                      hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                launch_dia_round(g->cap, bb);
                ok = hipStreamEndCapture(g->cap, &gr) == hipSuccess && gr != nullptr;
            }
            ok = ok && hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (gr) (void)hipGraphDestroy(gr);
            (void)hipGetLastError();
            if (!ok) {
                g->exec = nullptr;
                g->failed = true;
            } else {
                g->key = bb;
            }
        }
        if (g->exec && hipGraphLaunch(g->exec, ch.s) == hipSuccess) return;
        (void)hipGetLastError();
    }
    launch_dia_round(ch.s, bb);
}

void dia_graph_free(Chan &ch)
{
    if (!ch.dia) return;
    if (ch.dia->exec) (void)hipGraphExecDestroy(ch.dia->exec);
    if (ch.dia->cap) (void)hipStreamDestroy(ch.dia->cap);
    delete ch.dia;
    ch.dia = nullptr;
}

struct mpcg_ctx {
    int device = 0;
    int num_cu = 256;
    hipStream_t stream = nullptr;
    hipStream_t side_stream = nullptr;   // owned: the 2BFS of Algorithm II runs here
    Chan main, side;
    mpcg_options opt{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    DevState *hst = nullptr;   // pinned: [0],[1],[2] main channel, [3],[4],[5] side channel
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t tm[8] = {};
    KnnModel model;
    bool has_model = false;
    float last_kernel_ms = 0.0f;
    bool force_csr = false;   // spmv_variant 3: always use the CSR-stream kernels
    mpcg::batch::Engine *eng = nullptr;   // batched engine (own thread and stream), if started
    std::string arch;         // GPU architecture name (e.g. gfx950), the tuning table's key
    mpcg::TuneTable table;    // mpcg_load_tuning
    bool has_explicit = false;
    mpcg_tuning explicit_t{}; // mpcg_set_tuning
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
    L.state = take(sizeof(DevState));
    L.part = take(sizeof(double) * 5 * (size_t)kMaxGrid);   // product partials (up to 3 per block), update partials (up to 2)
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
    L.q0 = take(sizeof(QEnt) * N);
    L.q1 = take(sizeof(QEnt) * N);
    L.label = take(sizeof(int32_t) * N);
    L.tarr = take(sizeof(int32_t) * N);
    L.best = take(sizeof(unsigned long long) * N);
    // SELL-64 copy: padding up to the same number of entries again is accepted
    const size_t nsl = (N + 63) / 64;
    L.sell_cap = 2 * (int64_t)M + 64 * 64;
    L.sell_wid = take(sizeof(int64_t) * nsl);
    L.sell_off = take(sizeof(int64_t) * (nsl + 1));
    L.sell_col = take(sizeof(int32_t) * (size_t)L.sell_cap);
    L.sell_v64 = take(sizeof(double) * (size_t)L.sell_cap);
    L.sell_v32 = take(sizeof(float) * (size_t)L.sell_cap);
    L.ingest_blk = take(sizeof(int32_t) * 3 * ((N + kBlock - 1) / kBlock + 1));
    L.snap32 = take(sizeof(float) * kNumEps * N);
    L.z32 = take(sizeof(float) * N);
    L.z64 = take(sizeof(double) * N);
    L.dg32 = take(sizeof(float) * N);
    L.dg64 = take(sizeof(double) * N);
    L.dia_bits = take(sizeof(uint32_t) * (((N + 31) / 32 + 2) * (3 + 2 * kDiaMax) + 2 * kDiaRing + 8 * kDiaPartMax));
    L.total = off;
    return L;
}

SpmvShape spmv_shape(int64_t n, int64_t nnz, int value_bytes, int num_cu)
{
    // rows per tile so that a tile's entries fill one LDS chunk on average
    const int64_t chunk = kLdsBytes / (2 * value_bytes);
    int64_t avg = n > 0 ? (nnz + n - 1) / n : 1;
    if (avg < 1) avg = 1;
    int64_t R = chunk / avg;
    R = (R / 32) * 32;
    if (R < 32) R = 32;
    if (R > kBlock) R = kBlock;
    SpmvShape sh;
    sh.n = (int32_t)n;
    sh.R = (int32_t)R;
    sh.ntiles = (int32_t)((n + R - 1) / R);
    int64_t g = (int64_t)kSpmvBlocksPerCu * num_cu;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g > sh.ntiles) g = sh.ntiles;
    sh.grid = (int32_t)(g < 1 ? 1 : g);
    return sh;
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
    double *sp = nullptr;   // partials written by the product kernels (up to 3 per block)
    double *up = nullptr;   // partials written by the update kernel (2 per block with Jacobi)
    int pc = 0;             // Jacobi-preconditioned stages
    int32_t band = 0;       // largest |i - j| over the stored entries
    float *z32 = nullptr, *dg32 = nullptr;
    double *z64 = nullptr, *dg64 = nullptr;
    SpmvShape sh32{}, sh64{};
    SellMat sell{};
    bool use_sell = false;
    int nup = 1;
    mpcg_tuning tune{};   // scheduling parameters resolved for this matrix
    char *ws = nullptr;
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

// Scheduling parameters for a matrix: mpcg_set_tuning's, else the table's
// entry for its class, else the defaults; the options' explicit product and
// 2BFS variants override them.
mpcg_tuning resolve_tuning(const mpcg_ctx *c, int64_t n, int64_t nnz, int64_t band)
{
    mpcg_tuning t = c->has_explicit ? c->explicit_t : tune_lookup(c->table, c->arch, c->num_cu, n, nnz, band);
    if (c->opt.spmv_variant == 1) t.sell_split = 0;
    if (c->opt.spmv_variant == 2) t.sell_split = 1;
    if (c->opt.bfs_mode == 1) t.bfs_persist = 0;
    if (c->opt.bfs_mode == 2) t.bfs_persist = 1;
    return t;
}

mpcg_status read_state(const Chan &ch, const Plan &p, DevState *out)
{
    HIPCHK(hipMemcpyAsync(ch.sync, p.st, sizeof(DevState), hipMemcpyDeviceToHost, ch.s));
    HIPCHK(hipStreamSynchronize(ch.s));
    *out = *ch.sync;
    return MPCG_OK;
}

mpcg_status read_state(mpcg_ctx *c, const Plan &p, DevState *out) { return read_state(c->main, p, out); }

// Validate A (and b) on the device, convert row pointers / cast values when
// asked, and read back the verdict before any result buffer is touched.
mpcg_status ingest(mpcg_ctx *c, const mpcg_csr *A, const double *b, bool need_val32, Plan *p,
                   bool want_diag = false)
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
    p->sp = p->at<double>(p->L.part);
    p->up = p->sp + 3 * kMaxGrid;
    p->pc = want_diag ? 1 : 0;
    p->z32 = p->at<float>(p->L.z32);
    p->z64 = p->at<double>(p->L.z64);
    p->dg32 = p->at<float>(p->L.dg32);
    p->dg64 = p->at<double>(p->L.dg64);
    int32_t *rp32 = A->row_ptr_is_i64 ? p->at<int32_t>(p->L.rp32) : nullptr;
    p->rp = A->row_ptr_is_i64 ? rp32 : static_cast<const int32_t *>(A->row_ptr);
    HIPCHK(hipMemsetAsync(p->st, 0, sizeof(DevState), c->stream));
    int64_t *soff = p->at<int64_t>(p->L.sell_off);
    const int nsl = (p->n + 63) / 64;
    launch_ingest_sell(c->stream, A->row_ptr, A->row_ptr_is_i64 ? 1 : 0, p->rp, rp32, A->col_idx, A->val, b,
                       p->n, A->nnz, p->at<int64_t>(p->L.sell_wid), soff, p->at<int32_t>(p->L.ingest_blk),
                       p->L.sell_cap, c->force_csr ? 0 : 1,
                       p->ws + p->L.sell_col, p->at<double>(p->L.sell_v64),
                       need_val32 ? p->at<float>(p->L.sell_v32) : nullptr, p->st);
    if (want_diag) launch_diag(c->stream, p->rp, A->col_idx, A->val, p->n, p->dg64, p->dg32, p->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&c->hst[2].spare_i64, soff + nsl, sizeof(int64_t), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(&c->hst[1], p->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const DevState s = c->hst[1];
    const int64_t padded = c->hst[2].spare_i64;
    p->band = s.max_band;
    if (s.ing_err & (kErrRowPtr | kErrCol | kErrUnsorted)) return MPCG_EINVAL;
    if (s.ing_err & (kErrNonFiniteA | kErrNonFiniteB)) return MPCG_ENONFINITE;
    if (s.ing_err & kErrDiag) return MPCG_ENOTSPD;   // Jacobi needs a positive diagonal (any SPD A has one)
    // the entry kernel filled the SELL copy under exactly this condition
    p->use_sell = !c->force_csr && padded <= p->L.sell_cap;
    p->sh64 = spmv_shape(A->n, A->nnz, 8, c->num_cu);
    p->sh32 = spmv_shape(A->n, A->nnz, 4, c->num_cu);
    p->nup = vec_grid(A->n);
    if (p->nup > kUpdateGrid) p->nup = kUpdateGrid;
    p->tune = resolve_tuning(c, A->n, A->nnz, s.max_band);
    if (p->use_sell) {
        SellMat &m = p->sell;
        m.rp = p->rp;
        m.off = soff;
        m.n = p->n;
        m.nslices = nsl;
        m.idx16 = s.max_band < 32768 ? 1 : 0;
        m.batch = p->tune.sell_batch;
        m.bf_mask = p->tune.sell_whole_batch;
        // nontemporal matrix loads: where that precision's copy (values and
        // column offsets) exceeds the Infinity Cache, unless the tuning says
        const int64_t ib = m.idx16 ? 2 : 4;
        const int nt_auto = (padded * (8 + ib) > kInfinityCacheBytes ? 2 : 0) |
                            (padded * (4 + ib) > kInfinityCacheBytes ? 1 : 0);
        m.nt_mask = p->tune.sell_stream < 0 ? nt_auto : (p->tune.sell_stream ? 3 : 0);
        // scattered gathers (columns beyond 16-bit offsets): one gathered vector, not two
        m.split = p->tune.sell_split >= 0 ? p->tune.sell_split : (m.idx16 ? 0 : 1);
        int64_t g = ((int64_t)nsl + kBlock / 64 - 1) / (kBlock / 64);
        if (g > kMaxGrid) g = kMaxGrid;
        m.grid = (int32_t)(g < 1 ? 1 : g);
        m.scol = p->ws + p->L.sell_col;
        m.v64 = p->at<double>(p->L.sell_v64);
        m.v32 = need_val32 ? p->at<float>(p->L.sell_v32) : nullptr;
    } else if (need_val32) {
        launch_cast32(c->stream, A->val, p->at<float>(p->L.val32), A->nnz);
    }
    HIPCHK(hipGetLastError());
    return MPCG_OK;
}

// ---- dispatch: SELL-64 kernels when the padded copy fits, CSR-stream otherwise

int prod_grid(const Plan &p, bool f32) { return p.use_sell ? p.sell.grid : (f32 ? p.sh32.grid : p.sh64.grid); }

template <typename T> const T *csr_vals(const Plan &p);
template <> const float *csr_vals<float>(const Plan &p) { return p.at<float>(p.L.val32); }
template <> const double *csr_vals<double>(const Plan &p) { return p.val; }
template <typename T> const SpmvShape &csr_shape(const Plan &p);
template <> const SpmvShape &csr_shape<float>(const Plan &p) { return p.sh32; }
template <> const SpmvShape &csr_shape<double>(const Plan &p) { return p.sh64; }

template <typename T> T *snap_buf(const Plan &p);
template <> float *snap_buf<float>(const Plan &p) { return p.at<float>(p.L.snap32); }
template <> double *snap_buf<double>(const Plan &) { return nullptr; }

template <typename T> T *zbuf(const Plan &p);
template <> float *zbuf<float>(const Plan &p) { return p.z32; }
template <> double *zbuf<double>(const Plan &p) { return p.z64; }
template <typename T> const T *dgbuf(const Plan &p);
template <> const float *dgbuf<float>(const Plan &p) { return p.dg32; }
template <> const double *dgbuf<double>(const Plan &p) { return p.dg64; }

// The direction is built from r, or from z = M^-1 r with Jacobi.  snap is used
// only by the Algorithm II run-ahead (FP32).
template <typename T>
void run_cg_spmv(hipStream_t s, const Plan &p, const T *r, T *dA, T *dB, T *q, int it, int it0, T *x,
                 T *snap = nullptr)
{
    const T *src = p.pc ? zbuf<T>(p) : r;
    if (p.use_sell)
        launch_sell_cg_spmv<T>(s, p.sell, src, dA, dB, q, p.up, p.nup, p.sp, it, it0, x, snap, p.pc, p.st);
    else
        launch_cg_spmv<T>(s, csr_shape<T>(p), p.rp, p.col, csr_vals<T>(p), src, dA, dB, q, p.up, p.nup, p.sp,
                          it, it0, x, snap, p.pc, p.st);
}

template <typename T>
void run_cg_update(hipStream_t s, const Plan &p, T *r, const T *q, int it)
{
    launch_cg_update<T>(s, p.n, r, q, p.sp, prod_grid(p, sizeof(T) == 4), p.up, p.nup, it,
                        p.pc ? dgbuf<T>(p) : nullptr, p.pc ? zbuf<T>(p) : nullptr, p.st);
}

void run_restart(hipStream_t s, const Plan &p, const float *x32, double *x, const double *b, double *r,
                 double *dA, double *dB, int it0, double eps, int abs_tol, int32_t maxit)
{
    const double *dg = p.pc ? p.dg64 : nullptr;
    double *z = p.pc ? p.z64 : nullptr;
    if (p.use_sell) {
        launch_sell_restart(s, p.sell, x32, x, b, r, dA, dB, it0, dg, z, p.sp, p.st);
        launch_fin_restart(s, p.sp, p.sell.grid, it0, eps, abs_tol, maxit, p.st);
    } else {
        launch_restart(s, p.sh64, p.rp, p.col, p.val, x32, x, b, r, dA, dB, it0, eps, abs_tol, maxit, dg, z,
                       p.sp, p.st);
    }
}

void run_resid(hipStream_t s, const Plan &p, const double *x, const double *b)
{
    if (p.use_sell) {
        launch_sell_resid(s, p.sell, x, b, p.sp, p.st);
        launch_fin_resid(s, p.sp, p.sell.grid, p.st);
    } else {
        launch_resid(s, p.sh64, p.rp, p.col, p.val, x, b, p.sp, p.st);
    }
}

template <typename T>
void run_plain(hipStream_t s, const Plan &p, const T *x, T *y)
{
    if (p.use_sell) launch_sell_plain<T>(s, p.sell, x, y);
    else launch_spmv_plain<T>(s, csr_shape<T>(p), p.rp, p.col, csr_vals<T>(p), x, y);
}

int poll_iters(const mpcg_ctx *c) { return c->opt.graph_iters > 0 ? c->opt.graph_iters : 8; }

// Run CG iterations in precision T from iteration `it` (phase started at
// `it0`) until the device says stop, or until *stop_flag is set (Algorithm II
// run-ahead).  Groups of iterations are enqueued one ahead of the state
// snapshot being inspected; iterations enqueued after a device stop return at
// once.  *it_next gets the index of the next iteration that was not enqueued.
template <typename T>
mpcg_status cg_loop(mpcg_ctx *c, const Plan &p, T *x, T *r, T *q, T *dA, T *dB, int it, int it0,
                    DevState *out, const std::atomic<int> *stop_flag = nullptr, int *it_next = nullptr)
{
    const int G = poll_iters(c);
    const Chan &ch = c->main;
    T *snap = stop_flag ? snap_buf<T>(p) : nullptr;
    int64_t k = 0;
    for (;;) {
        for (int g = 0; g < G; ++g, ++it) {
            run_cg_spmv<T>(ch.s, p, r, dA, dB, q, it, it0, x, snap);
            run_cg_update<T>(ch.s, p, r, q, it);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ch.poll[k & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost, ch.s));
        HIPCHK(hipEventRecord(ch.ev[k & 1], ch.s));
        if (k > 0) {
            HIPCHK(hipEventSynchronize(ch.ev[(k - 1) & 1]));
            if (!ch.poll[(k - 1) & 1]->live) break;
        }
        if (stop_flag && stop_flag->load()) break;
        ++k;
        if (it > 0x7ffffff0 - G) return MPCG_EDEVICE;
    }
    if (it_next) *it_next = it;
    return read_state(ch, p, out);
}

// ---- two-stage Jacobi iteration

JacMat jac_mat(const Plan &p)
{
    JacMat m{};
    m.rp = p.rp;
    m.col = p.col;
    m.n = p.n;
    m.use_sell = p.use_sell;
    m.sell = p.sell;
    return m;
}

// One stage: Jacobi iterations from x0 until the device stops the stage;
// *out gets the state (iter = updates applied; the iterate is in x0 when iter
// is even, else in x1).
template <typename T>
mpcg_status jacobi_stage(mpcg_ctx *c, const Plan &p, const T *b, const T *dg, T *x0, T *x1, double eps,
                         int abs_tol, int32_t maxit, const double *b64, DevState *out)
{
    const JacMat m = jac_mat(p);
    const Chan &ch = c->main;
    launch_jacobi_begin(ch.s, m, b64, p.sp, p.st);
    const int G = poll_iters(c);
    int it = 0;
    for (int64_t g = 0;; ++g) {
        for (int j = 0; j < G; ++j, ++it)
            launch_jacobi_iter<T>(ch.s, m, csr_vals<T>(p), b, dg, x0, x1, it, maxit, eps, abs_tol, p.sp, p.st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ch.poll[g & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost, ch.s));
        HIPCHK(hipEventRecord(ch.ev[g & 1], ch.s));
        if (g > 0) {
            HIPCHK(hipEventSynchronize(ch.ev[(g - 1) & 1]));
            if (!ch.poll[(g - 1) & 1]->live) break;
        }
        if (it > 0x7ffffff0 - G) return MPCG_EDEVICE;
    }
    return read_state(ch, p, out);
}


BfsBufs bfs_bufs(const Plan &p, bool shared = false)
{
    BfsBufs b{};
    b.persist = p.tune.bfs_persist;
    b.grid = shared ? p.tune.bfs_grid_shared : p.tune.bfs_grid;
    b.precheck = 0;
    b.rp = p.rp;
    b.col = p.col;
    b.n = p.n;
    const int64_t avg = (p.nnz + p.n - 1) / p.n;
    int lanes = 1;
    while (lanes < avg && lanes < 32) lanes <<= 1;
    b.lanes = lanes;
    b.band = p.band;
    b.small_max = kBfsSmallWork / lanes;
    if (b.small_max < 64) b.small_max = 64;
    if (b.small_max > kBfsSmallCap) b.small_max = kBfsSmallCap;
    b.dia = 0;   // set by dia_prepare when the pattern qualifies
    b.nwords = (p.n + 31) / 32;
    b.dia_grid = kDiaPartMax;   // one word per thread: the level is latency-bound per word
    b.doff = DiaOffs{};
    {
        const size_t nw = (size_t)b.nwords + 2;
        uint32_t *bits = p.at<uint32_t>(p.L.dia_bits);
        b.df0 = bits;
        b.df1 = bits + nw;
        b.dv = bits + 2 * nw;
        b.dm = bits + 3 * nw;   // kDiaMax masks, b.nwords words apart
        b.draw = bits + 3 * nw + (size_t)kDiaMax * b.nwords;   // and their unaligned row masks
        int32_t *ring = reinterpret_cast<int32_t *>(b.draw + (size_t)kDiaMax * b.nwords);
        b.ring_cnt = ring;
        b.ring_min = ring + kDiaRing;
        b.part_cnt = ring + 2 * kDiaRing;
        b.part_min = ring + 2 * kDiaRing + 4 * kDiaPartMax;
    }
    b.dia_h = 0;
    b.dia_two = 0;
    b.dist = p.at<int32_t>(p.L.dist);
    b.q0 = p.at<QEnt>(p.L.q0);
    b.q1 = p.at<QEnt>(p.L.q1);
    b.label = p.at<int32_t>(p.L.label);
    b.tarr = p.at<int32_t>(p.L.tarr);
    b.best = p.at<unsigned long long>(p.L.best);
    b.st = p.st;
    return b;
}

// The bit-parallel levels over diagonals replace the queue kernels for a
// sweep when the tuning asks for them (bfs_dia: 1 on patterns wider than the
// one-workgroup kernel's narrow-band window, above 2^16 rows; 2 whenever it
// qualifies) and the pattern lies on at most kDiaMax diagonals.  Returns
// MPCG_OK whether or not it qualifies (bb->dia says which).
mpcg_status dia_prepare(const Chan &ch, const Plan &p, BfsBufs *bb)
{
    bb->dia = 0;
    const int mode = p.tune.bfs_dia;
    // launch k expands level k: at most n levels, kept below the launch index wrap
    if (mode == 0 || p.n >= (1 << 30) - 64 || (mode == 1 && (p.band <= 8 || p.n < (1 << 16)))) return MPCG_OK;
    launch_dia_detect(ch.s, *bb);
    HIPCHK(hipGetLastError());
    DevState s;
    mpcg_status rc = read_state(ch, p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.dia_over || s.dia_off[0] == 0) return MPCG_OK;
    bb->doff.nd = 0;
    for (int t = 0; t < kDiaMax && s.dia_off[t] != 0; ++t) bb->doff.d[bb->doff.nd++] = s.dia_off[t];
    for (int t = 0; t < kDiaMax; ++t) {
        if (t >= bb->doff.nd) bb->doff.d[t] = 0;
        const int64_t m = -(int64_t)bb->doff.d[t];
        bb->doff.q[t] = (int32_t)(m >= 0 ? m / 32 : -((-m + 31) / 32));   // floor(-d / 32)
        bb->doff.r[t] = (int32_t)(m - 32 * (int64_t)bb->doff.q[t]);
    }
    launch_dia_masks(ch.s, *bb);
    HIPCHK(hipGetLastError());
    bb->dia = 1;
    // temporal tiles: a tile's loaded range (kDiaTileWords) holds its own
    // words and a halo of h R words on each side; h as large as keeps the
    // own words at least half the range
    int R = 1;
    for (int t = 0; t < bb->doff.nd; ++t) {
        const int d = bb->doff.d[t] < 0 ? -bb->doff.d[t] : bb->doff.d[t];
        if (d / 32 + 1 > R) R = d / 32 + 1;
    }
    bb->dia_R = R;
    bb->dia_h = 0;
    // Tiles pay when a launch forms many levels over several tiles: a tile's
    // level runs on one CU, the per-level kernel's on the whole grid.
    if (p.tune.bfs_dia_tiles && bb->doff.nd <= kDiaTileDiags && R <= kDiaPad && bb->nwords > kDiaTileWords) {
        int h = kDiaTileWords / (4 * R);
        if (h > kDiaMaxLevels) h = kDiaMaxLevels;
        if (h >= kDiaTileMinLevels) {
            bb->dia_h = h;
            bb->dia_T = kDiaTileWords - 2 * h * R;
        }
    }
    // otherwise two levels per launch (chunks with a 2R-word halo in LDS)
    bb->dia_two = p.tune.bfs_dia_tiles && bb->dia_h == 0 && bb->doff.nd <= kDiaTileDiags && R <= kDia2MaxReach;
    return MPCG_OK;
}

mpcg_status bfs_run(const Chan &ch, const Plan &p, const BfsBufs &bb, DevState *out)
{
    if (bb.dia && bb.dia_h > 0) {   // temporal tiles: dia_h levels per launch
        const int launches = 64 / bb.dia_h > 1 ? 64 / bb.dia_h : 1;
        int k = 0;
        for (int64_t round = 0;; ++round) {
            k = launch_dia_multi_round(ch.s, bb, launches, k);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(ch.poll[round & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost, ch.s));
            HIPCHK(hipEventRecord(ch.ev[round & 1], ch.s));
            if (round > 0) {
                HIPCHK(hipEventSynchronize(ch.ev[(round - 1) & 1]));
                if (ch.poll[(round - 1) & 1]->bfs_done) break;
                if (ch.poll[(round - 1) & 1]->guard) {
                    (void)hipStreamSynchronize(ch.s);
                    return MPCG_EDEVICE;
                }
            }
            if (round > (int64_t)p.n + 4) return MPCG_EDEVICE;
        }
        return read_state(ch, p, out);
    }
    const int levels = 16;
    int k = 0;
    for (int64_t round = 0;; ++round) {
        if (bb.dia) dia_round(ch, bb);
        else k = launch_bfs_round(ch.s, bb, levels, k);
        if (k > 0x3fffffff) k &= 1;   // k only selects a parity slot: keep its parity
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ch.poll[round & 1], p.st, sizeof(DevState), hipMemcpyDeviceToHost, ch.s));
        HIPCHK(hipEventRecord(ch.ev[round & 1], ch.s));
        if (round > 0) {
            HIPCHK(hipEventSynchronize(ch.ev[(round - 1) & 1]));
            if (ch.poll[(round - 1) & 1]->bfs_done) break;
            if (ch.poll[(round - 1) & 1]->guard) {
                (void)hipStreamSynchronize(ch.s);
                return MPCG_EDEVICE;
            }
        }
        if (round > (int64_t)p.n + 4) return MPCG_EDEVICE;   // every round expands >= 1 level
    }
    return read_state(ch, p, out);
}

// 2BFS per component; fills pdiam, bfs_t, bfs_u, n_components.
mpcg_status pseudo_diameter_with(const Chan &ch, const Plan &p, BfsBufs bb, mpcg_features_t *f, int *dia_used)
{
    DevState s;
    *dia_used = 0;
    mpcg_status rc = dia_prepare(ch, p, &bb);
    if (rc != MPCG_OK) return rc;
    auto seed = [&](int32_t v) {
        if (bb.dia) {
            launch_dia_seed(ch.s, bb, v);
            launch_dia_ring_seed(ch.s, bb, v);
        } else {
            launch_bfs_seed_single(ch.s, bb, v);
        }
    };
    seed(0);
    rc = bfs_run(ch, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    if (s.guard) return MPCG_EDEVICE;
    if (s.bfs_visited == p.n) {
        const int32_t t = s.bfs_far;
        seed(t);
        rc = bfs_run(ch, p, bb, &s);
        if (rc != MPCG_OK) return rc;
        f->pdiam = s.bfs_ecc;
        f->bfs_t = t;
        f->bfs_u = s.bfs_far;
        f->n_components = 1;
        *dia_used = bb.dia;
        return MPCG_OK;
    }
    bb.dia = 0;   // not connected: components and multi-source sweeps on the queue kernels
    launch_cc(ch.s, bb);
    launch_bfs_seed_roots(ch.s, bb);
    rc = bfs_run(ch, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    launch_comp_argmax(ch.s, bb, 0);
    launch_bfs_seed_far(ch.s, bb);
    rc = bfs_run(ch, p, bb, &s);
    if (rc != MPCG_OK) return rc;
    launch_comp_argmax(ch.s, bb, 1);
    launch_comp_final(ch.s, bb);
    HIPCHK(hipGetLastError());
    rc = read_state(ch, p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.guard) return MPCG_EDEVICE;
    const uint64_t key = s.comp_best;
    const int32_t comp = (int32_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
    int32_t t = 0;
    unsigned long long bu = 0;
    HIPCHK(hipMemcpyAsync(&t, bb.tarr + comp, sizeof(int32_t), hipMemcpyDeviceToHost, ch.s));
    HIPCHK(hipMemcpyAsync(&bu, bb.best + comp, sizeof(bu), hipMemcpyDeviceToHost, ch.s));
    HIPCHK(hipStreamSynchronize(ch.s));
    f->pdiam = (int64_t)(key >> 32);
    f->bfs_t = t;
    f->bfs_u = (int64_t)(0xffffffffu - (uint32_t)(bu & 0xffffffffull));
    f->n_components = s.ncomp;
    return MPCG_OK;
}

// The persistent level kernel bounds its barrier waits; if one ran out (its
// blocks could not all be resident), the BFS is repeated with one launch per
// level, which needs no co-residency.
// *dia_used (if given): both sweeps ran as bit-parallel levels over diagonals.
mpcg_status pseudo_diameter(const mpcg_ctx *c, const Chan &ch, const Plan &p, mpcg_features_t *f,
                            bool shared = false, int *dia_used = nullptr)
{
    BfsBufs bb = bfs_bufs(p, shared);
    int dia = 0;
    mpcg_status rc = pseudo_diameter_with(ch, p, bb, f, &dia);
    if (rc == MPCG_EDEVICE && bb.persist) {
        HIPCHK(hipStreamSynchronize(ch.s));
        HIPCHK(hipMemsetAsync(&p.st->guard, 0, sizeof(int32_t), ch.s));
        bb.persist = 0;
        rc = pseudo_diameter_with(ch, p, bb, f, &dia);
    }
    if (dia_used) *dia_used = dia;
    return rc;
}

// The plan of the FP32 launches that run beside the 2BFS: when the SELL
// product grid fills every CU (8 blocks of 256 threads each), one block per CU
// fewer.  Both kernels of an iteration take their partial counts from the
// same plan, and the first product after the switch reduces the update's
// partials, whose grid does not change.
Plan shared_plan(const mpcg_ctx *c, const Plan &p)
{
    Plan q = p;
    if (p.use_sell && p.sell.grid >= 8 * c->num_cu) {
        const int g = 7 * c->num_cu;
        if (g < q.sell.grid) q.sell.grid = g;
    }
    return q;
}

// FP32 prefix of Algorithm II: k0 iterations without the eps1 test.
mpcg_status fp32_prefix(mpcg_ctx *c, const Plan &p, const double *b, int32_t k0, DevState *s)
{
    float *x = p.at<float>(p.L.x32), *r = p.at<float>(p.L.r32), *q = p.at<float>(p.L.q32);
    float *dA = p.at<float>(p.L.dA32), *dB = p.at<float>(p.L.dB32);
    // thr = 0: only gamma' = 0 or a breakdown ends the prefix before k0
    launch_init32(c->stream, b, x, r, dA, p.n, 0.0, 1, k0, k0, p.pc ? p.dg32 : nullptr, p.z32, p.sp, p.st,
                  c->opt.dot_acc);
    HIPCHK(hipGetLastError());
    mpcg_status rc = read_state(c, p, s);
    if (rc != MPCG_OK) return rc;
    if (s->live) rc = cg_loop<float>(c, p, x, r, q, dA, dB, 0, 0, s);
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
    if (o.k0 > kK0Max || o.tol_mode < 0 || o.tol_mode > 1 || o.knn_k < 0 || o.graph_iters < 0 ||
        o.precond < 0 || o.precond > 1 || o.dot_acc < 0 || o.dot_acc > 1 || o.spmv_variant < 0 ||
        o.spmv_variant > 3 || o.bfs_mode < 0 || o.bfs_mode > 2)
        return MPCG_EINVAL;
    mpcg_ctx *c = new (std::nothrow) mpcg_ctx();
    if (!c) return MPCG_EDEVICE;
    c->opt = o;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->force_csr = o.spmv_variant == 3;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&c->device) != hipSuccess || scratch_init(c->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipHostMalloc((void **)&c->hst, 6 * sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess) {
        mpcg_destroy(c);
        return MPCG_EDEVICE;
    }
    {
        const std::string name(prop.gcnArchName);
        c->arch = name.substr(0, name.find(':'));   // "gfx950:sramecc+:xnack-" -> "gfx950"
    }
    for (auto &e : c->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { mpcg_destroy(c); return MPCG_EDEVICE; }
    for (auto &e : c->tm)
        if (hipEventCreate(&e) != hipSuccess) { mpcg_destroy(c); return MPCG_EDEVICE; }
    c->main.s = c->stream;
    c->main.poll[0] = &c->hst[0];
    c->main.poll[1] = &c->hst[1];
    c->main.sync = &c->hst[2];
    c->main.ev[0] = c->ev[0];
    c->main.ev[1] = c->ev[1];
    c->main.dia = new (std::nothrow) DiaGraph();   // null: plain launches
    c->side.dia = new (std::nothrow) DiaGraph();
    c->side.s = c->side_stream;
    c->side.poll[0] = &c->hst[3];
    c->side.poll[1] = &c->hst[4];
    c->side.sync = &c->hst[5];
    for (auto &e : c->side.ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { mpcg_destroy(c); return MPCG_EDEVICE; }
    *out = c;
    return MPCG_OK;
}

mpcg_status mpcg_destroy(mpcg_ctx *c)
{
    if (!c) return MPCG_EINVAL;
    if (c->eng) mpcg::batch::engine_destroy(c->eng);
    (void)hipStreamSynchronize(c->stream);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    dia_graph_free(c->main);
    dia_graph_free(c->side);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->side.ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->tm) if (e) (void)hipEventDestroy(e);
    if (c->hst) (void)hipHostFree(c->hst);
    knn_free(&c->model);
    delete c;
    return MPCG_OK;
}

mpcg_status mpcg_set_tuning(mpcg_ctx *c, const mpcg_tuning *t)
{
    if (!c) return MPCG_EINVAL;
    if (!t) {
        c->has_explicit = false;
        return MPCG_OK;
    }
    if (!tune_valid(*t)) return MPCG_EINVAL;
    c->explicit_t = *t;
    c->has_explicit = true;
    return MPCG_OK;
}

mpcg_status mpcg_load_tuning(mpcg_ctx *c, const char *path)
{
    if (!c || !path) return MPCG_EINVAL;
    TuneTable tb;
    if (tune_load(path, &tb) != 0) return MPCG_EINVAL;
    c->table = tb;
    return MPCG_OK;
}

mpcg_status mpcg_get_tuning(const mpcg_ctx *c, int64_t n, int64_t nnz, int64_t band, mpcg_tuning *out)
{
    if (!c || !out || n <= 0 || nnz < 0 || band < 0) return MPCG_EINVAL;
    *out = resolve_tuning(c, n, nnz, band);
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
    mpcg_status rc = ingest(c, A, b, true, &p, c->opt.precond == 1);
    if (rc != MPCG_OK) return rc;
    mpcg_features_t f{};
    f.n = A->n;
    f.m = A->nnz;
    rc = pseudo_diameter(c, c->main, p, &f);
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
    mpcg_status rc = ingest(c, A, b, !dponly, &p, c->opt.precond == 1);
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
    bool spec_final = false;      // the FP64 phase is the speculative one (its restart residual below)
    double spec_rr_final = 0.0;

    if (!dponly) {
        float *x32 = p.at<float>(p.L.x32), *r32 = p.at<float>(p.L.r32), *q32 = p.at<float>(p.L.q32);
        float *dA32 = p.at<float>(p.L.dA32), *dB32 = p.at<float>(p.L.dB32);
        const float *x32_src = x32;   // x~ handed to the FP64 restart
        bool broke = false;
        // speculative FP64 phase (below): started from the tightest candidate's
        // state when the run-ahead has crossed every candidate before the
        // features are in; kept if the kNN chooses that candidate
        bool spec64 = false, spec_keep = false;
        DevState s64{};
        int it64_next = 0;
        double spec_rr = 0.0;
        if (autoe) {
            // Algorithm II.  The 2BFS runs on the side stream from a host
            // thread.  Meanwhile the main stream does the k0-iteration prefix
            // (v) and then keeps iterating the same FP32 recurrence, copying x~
            // the first time sqrt(gamma) drops below each candidate eps1 * ||b||.
            // Once kNN has chosen eps1 the state at that first crossing -- the
            // state Algorithm II stops in -- is taken from its copy.
            mpcg_features_t f{};
            f.n = n;
            f.m = A->nnz;
            mpcg_status rc_bfs = MPCG_OK;
            int bfs_dia = 0;
            std::atomic<int> bfs_done{0};
            std::thread bfs_thread([&]() {
                (void)hipSetDevice(c->device);
                (void)hipEventRecord(c->tm[1], c->side.s);
                rc_bfs = pseudo_diameter(c, c->side, p, &f, true, &bfs_dia);
                (void)hipEventRecord(c->tm[2], c->side.s);
                (void)hipEventSynchronize(c->tm[2]);
                bfs_done.store(1);
            });
            const Plan ps = shared_plan(c, p);   // FP32 launches beside the BFS
            DevState sp0;
            rc = fp32_prefix(c, ps, b, c->opt.k0, &sp0);
            s = sp0;
            int it_next = sp0.iter;
            broke = (sp0.reason == kNotSpd || sp0.reason == kNonFinite);
            if (rc == MPCG_OK && sp0.bnorm2 > 0.0 && !broke) {
                launch_set_spec(c->stream, p.st, abs_tol ? 1.0 : std::sqrt(sp0.bnorm2), sp0.iter, maxit1);
                rc = cg_loop<float>(c, ps, x32, r32, q32, dA32, dB32, sp0.iter, 0, &s, &bfs_done, &it_next);
                if (rc == MPCG_OK && !s.live && s.reason == kConverged && s.cross_iter[kNumEps - 1] >= 0 &&
                    !bfs_done.load()) {
                    // every candidate crossed and the features still pending: x~ is
                    // the state Algorithm II restarts from if the kNN picks the
                    // tightest candidate, so that FP64 phase starts now (beside
                    // the BFS); another choice discards it and restarts from its copy
                    HIPCHK(hipEventRecord(c->tm[3], c->stream));
                    run_restart(c->stream, ps, x32, x, b, r64, dA64, dB64, 0, eps2, abs_tol, maxit2);
                    HIPCHK(hipGetLastError());
                    rc = read_state(c, p, &s64);
                    if (rc == MPCG_OK) {
                        spec64 = true;
                        spec_rr = s64.bnorm2 > 0.0 ? std::sqrt(s64.gamma) / std::sqrt(s64.bnorm2) : 0.0;
                        it64_next = s64.iter;
                        if (s64.live)
                            rc = cg_loop<double>(c, ps, x, r64, q64, dA64, dB64, s64.iter, 0, &s64, &bfs_done,
                                                 &it64_next);
                    }
                }
            }
            bfs_thread.join();
            if (rc == MPCG_OK) rc = rc_bfs;
            if (rc != MPCG_OK) { S.status = rc; if (stats) *stats = S; return rc; }
            feat_timed = true;
            if (sp0.bnorm2 == 0.0) goto zero_rhs;
            f.k0_used = sp0.iter;
            f.v = v_from_ratios(sp0, sp0.iter);
            S.feat = f;
            const double chi[4] = {(double)f.n, (double)f.m, (double)f.pdiam, f.v};
            int32_t exact = 0;
            const int cls = knn_select(c->model, chi, c->opt.knn_k, &exact);
            if (cls < 2 || cls > 7) { S.status = MPCG_EINVAL; if (stats) *stats = S; return MPCG_EINVAL; }
            const double e1 = kEpsClass[cls];
            S.eps1_class = cls;
            S.eps1_used = e1;
            if (exact) S.flags |= MPCG_FLAG_KNN_EXACT;
            if (bfs_dia) S.flags |= MPCG_FLAG_BFS_DIA;
            spec_keep = spec64 && cls - 2 == kNumEps - 1;
            if (!broke) {
                const int ci = cls - 2;
                if (s.cross_iter[ci] >= 0) {
                    // crossed during the run-ahead: restart from the copy
                    x32_src = p.at<float>(p.L.snap32) + (size_t)ci * p.n;
                    s.iter = s.cross_iter[ci];
                    s.gamma = s.cross_gamma[ci];
                    s.reason = kConverged;
                } else if (s.live) {
                    // not there yet: continue with the chosen tolerance (Remark 3)
                    const double thr1 = abs_tol ? e1 : e1 * std::sqrt(sp0.bnorm2);
                    launch_set_phase(c->stream, p.st, thr1, maxit1, c->opt.k0);
                    HIPCHK(hipGetLastError());
                    rc = cg_loop<float>(c, p, x32, r32, q32, dA32, dB32, it_next, 0, &s);
                    if (rc != MPCG_OK) return rc;
                }
                // otherwise the run-ahead stopped (breakdown or maxit1) before
                // reaching eps1: s already holds that stop
            }
        } else {
            launch_init32(c->stream, b, x32, r32, dA32, p.n, eps1, abs_tol, maxit1, 0, p.pc ? p.dg32 : nullptr,
                          p.z32, p.sp, p.st, c->opt.dot_acc);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
            if (s.bnorm2 == 0.0) goto zero_rhs;
            if (s.live) rc = cg_loop<float>(c, p, x32, r32, q32, dA32, dB32, 0, 0, &s);
            if (rc != MPCG_OK) return rc;
        }
        if (s.reason == kNotSpd || s.reason == kNonFinite) S.flags |= MPCG_FLAG_FP32_BREAKDOWN;
        else if (s.reason == kMaxit) S.flags |= MPCG_FLAG_FP32_MAXIT;
        S.n1 = s.iter;
        bnorm = std::sqrt(s.bnorm2);
        S.relres_sp = std::sqrt(s.gamma) / bnorm;
        spec_final = spec_keep;
        spec_rr_final = spec_rr;
        if (spec_keep) {
            // the speculative FP64 phase is the chosen one: it continues
            if (s64.live) {
                rc = cg_loop<double>(c, p, x, r64, q64, dA64, dB64, it64_next, 0, &s64);
                if (rc != MPCG_OK) return rc;
            }
        } else {
            HIPCHK(hipEventRecord(c->tm[3], c->stream));
            // restart in FP64 from float64(x~) with a freshly computed residual
            run_restart(c->stream, p, x32_src, x, b, r64, dA64, dB64, 0, eps2, abs_tol, maxit2);
            HIPCHK(hipGetLastError());
        }
    } else {
        // FP64-only CG from x0 = 0 through the restart kernel: r = b - A*0 = b
        // exactly, with the same reductions as the mixed path's restart.
        HIPCHK(hipEventRecord(c->tm[3], c->stream));
        launch_fill_f64(c->stream, x, n, 0.0);
        run_restart(c->stream, p, nullptr, x, b, r64, dA64, dB64, 0, eps2, abs_tol, maxit2);
        HIPCHK(hipGetLastError());
    }
    rc = read_state(c, p, &s);
    if (rc != MPCG_OK) return rc;
    if (s.bnorm2 == 0.0) goto zero_rhs;
    bnorm = std::sqrt(s.bnorm2);
    S.relres_restart_true = std::sqrt(s.gamma) / bnorm;
    if (spec_final) S.relres_restart_true = spec_rr_final;
    {
        const double thr2 = abs_tol ? eps2 : eps2 * bnorm;
        for (;;) {
            if (s.live) {
                rc = cg_loop<double>(c, p, x, r64, q64, dA64, dB64, s.iter, s.iter, &s);
                if (rc != MPCG_OK) return rc;
            }
            if (s.reason == kMaxit) { rc = MPCG_ENOCONV; break; }
            if (s.reason == kNotSpd) { rc = MPCG_ENOTSPD; break; }
            if (s.reason == kNonFinite) { rc = MPCG_ENONFINITE; break; }
            run_resid(c->stream, p, x, b);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
            const double rho = std::sqrt(s.resid2);
            S.relres_final_true = rho / bnorm;
            if (rho <= thr2) { rc = MPCG_OK; break; }
            if (S.restarts >= c->opt.max_restarts) { rc = MPCG_ENOCONV; break; }
            S.restarts++;
            S.flags |= MPCG_FLAG_FINAL_RESTARTED;
            run_restart(c->stream, p, nullptr, x, b, r64, dA64, dB64, s.iter, eps2, abs_tol, maxit2);
            HIPCHK(hipGetLastError());
            rc = read_state(c, p, &s);
            if (rc != MPCG_OK) return rc;
        }
        if (rc != MPCG_OK && S.relres_final_true == 0.0) {
            run_resid(c->stream, p, x, b);
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
    // the 2BFS overlaps the FP32 phase (side stream), so t_sp_ms is the main
    // stream's time from the start of the call to the restart
    if (feat_timed) S.t_feat_ms = elapsed(c->tm[1], c->tm[2]);
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

mpcg_status mpcg_solve_noalloc(mpcg_ctx *c, const mpcg_csr *A, const double *b, double *x, double eps1,
                               double eps2, mpcg_stats *stats)
{
    if (!c || !A || A->n <= 0 || A->n >= 0x7fffffff || A->nnz < 0 || A->nnz >= 0x7fffffff) return MPCG_EINVAL;
    if (plan_layout(A->n, A->nnz).total > kNoAllocBytes) return MPCG_ENOMEM;
    void *ptr = scratch_of(c->device);
    if (!ptr) return MPCG_EDEVICE;
    // the solve runs on the device array instead of the context's arena; every
    // region the solve reads before writing is cleared by the solve itself
    char *const ws = c->ws;
    const size_t ws_bytes = c->ws_bytes;
    c->ws = static_cast<char *>(ptr);
    c->ws_bytes = kNoAllocBytes;
    if (c->main.dia) c->main.dia->suspended = true;
    if (c->side.dia) c->side.dia->suspended = true;
    const mpcg_status rc = mpcg_solve(c, A, b, x, eps1, eps2, stats);
    if (c->main.dia) c->main.dia->suspended = false;
    if (c->side.dia) c->side.dia->suspended = false;
    c->ws = ws;
    c->ws_bytes = ws_bytes;
    return rc;
}

mpcg_status mpcg_spmv(mpcg_ctx *c, const mpcg_csr *A, int32_t precision, const void *x, void *y)
{
    if (!c || !x || !y || (precision != 32 && precision != 64)) return MPCG_EINVAL;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, precision == 32, &p);
    if (rc != MPCG_OK) return rc;
    HIPCHK(hipEventRecord(c->tm[5], c->stream));
    if (precision == 64)
        run_plain<double>(c->stream, p, static_cast<const double *>(x), static_cast<double *>(y));
    else
        run_plain<float>(c->stream, p, static_cast<const float *>(x), static_cast<float *>(y));
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
    rc = dia_prepare(c->main, p, &bb);
    if (rc != MPCG_OK) return rc;
    auto seed = [&]() {
        if (bb.dia) {
            launch_dia_seed(c->stream, bb, (int32_t)src);
            launch_dia_ring_seed(c->stream, bb, (int32_t)src);
        } else {
            launch_bfs_seed_single(c->stream, bb, (int32_t)src);
        }
    };
    seed();
    DevState s;
    rc = bfs_run(c->main, p, bb, &s);
    if (rc == MPCG_EDEVICE && bb.persist) {   // see pseudo_diameter
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemsetAsync(&p.st->guard, 0, sizeof(int32_t), c->stream));
        bb.persist = 0;
        seed();
        rc = bfs_run(c->main, p, bb, &s);
    }
    if (rc != MPCG_OK) return rc;
    HIPCHK(hipMemcpyAsync(dist, bb.dist, sizeof(int32_t) * (size_t)p.n, hipMemcpyDeviceToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (ecc) *ecc = s.bfs_ecc;
    if (far) *far = s.bfs_far;
    return MPCG_OK;
}

mpcg_status mpcg_solve_jacobi(mpcg_ctx *c, const mpcg_csr *A, const double *b, double *x, double eps1,
                              double eps2, mpcg_stats *stats)
{
    if (!c || !A || !b || !x) return MPCG_EINVAL;
    if (!(eps2 > 0.0) || !std::isfinite(eps2)) return MPCG_EINVAL;
    const bool dponly = (eps1 == MPCG_EPS1_NONE);
    if (!dponly && !(eps1 > 0.0 && std::isfinite(eps1))) return MPCG_EINVAL;
    mpcg_stats S{};
    S.eps1_class = -1;
    S.eps1_used = dponly ? -1.0 : eps1;
    HIPCHK(hipEventRecord(c->tm[0], c->stream));
    Plan p;
    mpcg_status rc = ingest(c, A, b, !dponly, &p, true);
    if (rc != MPCG_OK) {
        S.status = rc;
        if (stats) *stats = S;
        return rc;
    }
    const int abs_tol = c->opt.tol_mode == 1;
    const int64_t n = A->n;
    int64_t mi1 = c->opt.maxit1 > 0 ? c->opt.maxit1 : n;
    int64_t mi2 = c->opt.maxit2 > 0 ? c->opt.maxit2 : (10 * n > 1000 ? 10 * n : 1000);
    const int32_t maxit1 = (int32_t)(mi1 < 0x7fff0000 ? mi1 : 0x7fff0000);
    const int32_t maxit2 = (int32_t)(mi2 < 0x7fff0000 ? mi2 : 0x7fff0000);
    DevState s;
    if (!dponly) {
        float *b32 = p.at<float>(p.L.r32);
        float *xa = p.at<float>(p.L.x32), *xb = p.at<float>(p.L.dA32);
        launch_cast32(c->stream, b, b32, n);
        launch_fill_f32(c->stream, xa, n, 0.0f);
        rc = jacobi_stage<float>(c, p, b32, p.dg32, xa, xb, eps1, abs_tol, maxit1, b, &s);
        if (rc != MPCG_OK) return rc;
        S.n1 = s.iter;
        if (s.reason == kMaxit) S.flags |= MPCG_FLAG_FP32_MAXIT;
        else if (s.reason == kNonFinite) S.flags |= MPCG_FLAG_FP32_BREAKDOWN;
        if (s.bnorm2 > 0.0) S.relres_sp = std::sqrt(s.gamma) / std::sqrt(s.bnorm2);
        launch_jacobi_widen(c->stream, (s.iter & 1) ? xb : xa, x, (int32_t)n);
    } else {
        launch_fill_f64(c->stream, x, n, 0.0);
    }
    HIPCHK(hipEventRecord(c->tm[3], c->stream));
    double *q64 = p.at<double>(p.L.q64);
    rc = jacobi_stage<double>(c, p, b, p.dg64, x, q64, eps2, abs_tol, maxit2, b, &s);
    if (rc != MPCG_OK) return rc;
    S.n2 = s.iter;
    if (s.iter & 1) HIPCHK(hipMemcpyAsync(x, q64, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipEventRecord(c->tm[4], c->stream));
    HIPCHK(hipEventSynchronize(c->tm[4]));
    S.relres_final_true = s.bnorm2 > 0.0 ? std::sqrt(s.gamma) / std::sqrt(s.bnorm2) : 0.0;
    const mpcg_status fin = s.reason == kConverged ? MPCG_OK : (s.reason == kNonFinite ? MPCG_ENONFINITE : MPCG_ENOCONV);
    S.status = fin;
    float t_sp = 0.f, t_dp = 0.f;
    (void)hipEventElapsedTime(&t_sp, c->tm[0], c->tm[3]);
    (void)hipEventElapsedTime(&t_dp, c->tm[3], c->tm[4]);
    S.t_sp_ms = t_sp;
    S.t_dp_ms = t_dp;
    S.t_total_ms = (double)t_sp + (double)t_dp;
    if (stats) *stats = S;
    return fin;
}

mpcg_status mpcg_diameter_multi(mpcg_ctx *c, const mpcg_csr *A, const int32_t *starts, int32_t count, double q,
                                mpcg_diam_t *out)
{
    if (!c || !A || !out || count < 0 || (count > 0 && !starts) || !(q > 0.0 && q <= 1.0)) return MPCG_EINVAL;
    for (int32_t i = 0; i < count; ++i)
        if (starts[i] < 0 || (int64_t)starts[i] >= A->n) return MPCG_EINVAL;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, false, &p);
    if (rc != MPCG_OK) return rc;
    mpcg_features_t f{};
    rc = pseudo_diameter(c, c->main, p, &f);
    if (rc != MPCG_OK) return rc;
    mpcg_diam_t d{};
    d.pdiam = f.pdiam;
    d.pdiam_multi = f.pdiam;
    d.best_start = -1;
    BfsBufs bb = bfs_bufs(p);
    bb.persist = 0;   // one launch per level: needs no co-residency
    // the per-component key array is not used by single-source sweeps
    unsigned long long *hist = bb.best;
    launch_fill_f64(c->stream, reinterpret_cast<double *>(hist), p.n, 0.0);
    int64_t max_ecc = 0;
    for (int32_t i = 0; i < count; ++i) {
        DevState s1, s2;
        launch_bfs_seed_single(c->stream, bb, starts[i]);
        rc = bfs_run(c->main, p, bb, &s1);
        if (rc != MPCG_OK) return rc;
        launch_dist_hist(c->stream, bb.dist, p.n, hist);
        if (s1.bfs_ecc > max_ecc) max_ecc = s1.bfs_ecc;
        launch_bfs_seed_single(c->stream, bb, s1.bfs_far);
        rc = bfs_run(c->main, p, bb, &s2);
        if (rc != MPCG_OK) return rc;
        if (s2.bfs_ecc > d.pdiam_multi) {
            d.pdiam_multi = s2.bfs_ecc;
            d.best_start = i;
        }
    }
    if (count > 0 && max_ecc > 0) {
        std::vector<unsigned long long> h((size_t)max_ecc + 1);
        HIPCHK(hipMemcpyAsync(h.data(), hist, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        unsigned long long total = 0, cum = 0;
        for (size_t k = 1; k < h.size(); ++k) total += h[k];
        d.pairs = (int64_t)total;
        for (size_t k = 1; k < h.size(); ++k) {
            cum += h[k];
            if ((double)cum >= q * (double)total) {
                d.eff_diam = (int64_t)k;
                break;
            }
        }
    }
    HIPCHK(hipGetLastError());
    *out = d;
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
    if (!c || !A || !ms || reps < 1 || kernel < 0 || kernel > 7) return MPCG_EINVAL;
    const bool f32 = (kernel & 1) != 0;
    const bool jac = kernel >= MPCG_KERNEL_JACOBI_F64;
    Plan p;
    mpcg_status rc = ingest(c, A, nullptr, f32, &p, jac);
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
    launch_timing_state(c->stream, p.st, p.sp, 5 * kMaxGrid);
    HIPCHK(hipGetLastError());
    auto one = [&]() {
        switch (kernel) {
        case MPCG_KERNEL_CG_SPMV_F64:
            run_cg_spmv<double>(c->stream, p, r64, dA64, dB64, q64, 1, 0, x64);
            break;
        case MPCG_KERNEL_CG_SPMV_F32:
            run_cg_spmv<float>(c->stream, p, r32, dA32, dB32, q32, 1, 0, x32);
            break;
        case MPCG_KERNEL_UPDATE_F64:
            run_cg_update<double>(c->stream, p, r64, q64, 1);
            break;
        case MPCG_KERNEL_UPDATE_F32:
            run_cg_update<float>(c->stream, p, r32, q32, 1);
            break;
        case MPCG_KERNEL_SPMV_F64:
            run_plain<double>(c->stream, p, r64, q64);
            break;
        case MPCG_KERNEL_JACOBI_F64:   // threshold 0 and no cap: every launch runs
            launch_jacobi_iter<double>(c->stream, jac_mat(p), csr_vals<double>(p), r64, p.dg64, x64, dA64, 1,
                                       0x7fff0000, 0.0, 1, p.sp, p.st);
            break;
        case MPCG_KERNEL_JACOBI_F32:
            launch_jacobi_iter<float>(c->stream, jac_mat(p), csr_vals<float>(p), r32, p.dg32, x32, dA32, 1,
                                      0x7fff0000, 0.0, 1, p.sp, p.st);
            break;
        default:
            run_plain<float>(c->stream, p, r32, q32);
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

// ------------------------------------------------------------- batches --

mpcg_status mpcg_batch_workspace_size(const mpcg_ctx *c, int64_t max_rows, int64_t max_entries,
                                      int32_t max_systems, size_t *bytes)
{
    if (!c || !bytes || max_rows <= 0 || max_entries <= 0 || max_systems <= 0 || max_systems > (1 << 16))
        return MPCG_EINVAL;
    const int64_t ms = (max_rows + 63) / 64;
    if (ms > 0x7fffffff / 64) return MPCG_EINVAL;
    *bytes = mpcg::batch::arena_bytes(max_systems, (int32_t)ms, max_entries);
    return MPCG_OK;
}

mpcg_status mpcg_batch_set_workspace(mpcg_ctx *c, void *arena, size_t bytes, int64_t max_rows,
                                     int64_t max_entries, int32_t max_systems)
{
    if (!c || !arena || ((uintptr_t)arena & 255)) return MPCG_EINVAL;
    if (c->opt.precond != 0) return MPCG_EINVAL;   // the batched engine runs unpreconditioned stages
    if (c->eng) return MPCG_EBUSY;
    int st = MPCG_OK;
    const mpcg_tuning bt = c->has_explicit ? c->explicit_t : tune_batch(c->table, c->arch, c->num_cu);
    c->eng = mpcg::batch::engine_create(c->device, c->opt, bt, &c->model, arena, bytes, max_rows, max_entries,
                                        max_systems, &st);
    return (mpcg_status)st;
}

mpcg_status mpcg_batch_submit(mpcg_ctx *c, const mpcg_request *reqs, int32_t count, uint64_t *ids)
{
    if (!c || count < 0 || (count > 0 && (!reqs || !ids))) return MPCG_EINVAL;
    if (!c->eng) return MPCG_EDEVICE;
    for (int32_t i = 0; i < count; ++i) {
        const mpcg_request &r = reqs[i];
        if (r.A.n <= 0 || r.A.n > 0x7fffffc0 || r.A.nnz < 0 || !r.A.row_ptr || !r.b || !r.x) return MPCG_EINVAL;
        if (r.A.nnz > 0 && (!r.A.col_idx || !r.A.val)) return MPCG_EINVAL;
        if (!(r.eps2 > 0.0) || !std::isfinite(r.eps2)) return MPCG_EINVAL;
        const bool autoe = r.eps1 == MPCG_EPS1_AUTO, none = r.eps1 == MPCG_EPS1_NONE;
        if (!autoe && !none && !(r.eps1 > 0.0 && std::isfinite(r.eps1))) return MPCG_EINVAL;
        if (autoe && (!c->has_model || c->model.ns <= 0)) return MPCG_ENOMODEL;
        if ((r.A.n + 63) / 64 > mpcg::batch::engine_max_slices(c->eng) ||
            r.A.nnz > mpcg::batch::engine_max_entries(c->eng))
            return MPCG_ENOMEM;
    }
    return (mpcg_status)mpcg::batch::engine_submit(c->eng, reqs, count, ids);
}

mpcg_status mpcg_batch_poll(mpcg_ctx *c, uint64_t *done_ids, mpcg_stats *done_stats, int32_t cap,
                            int32_t *n_done)
{
    if (!c || !n_done || cap < 0 || (cap > 0 && !done_ids)) return MPCG_EINVAL;
    if (!c->eng) return MPCG_EDEVICE;
    return (mpcg_status)mpcg::batch::engine_poll(c->eng, done_ids, done_stats, cap, n_done);
}

mpcg_status mpcg_batch_cancel(mpcg_ctx *c, uint64_t id)
{
    if (!c) return MPCG_EINVAL;
    if (!c->eng) return MPCG_EDEVICE;
    return (mpcg_status)mpcg::batch::engine_cancel(c->eng, id);
}

mpcg_status mpcg_batch_load(mpcg_ctx *c, int32_t *queued, int32_t *active)
{
    if (!c) return MPCG_EINVAL;
    if (!c->eng) return MPCG_EDEVICE;
    return (mpcg_status)mpcg::batch::engine_load(c->eng, queued, active);
}

}  // extern "C"
