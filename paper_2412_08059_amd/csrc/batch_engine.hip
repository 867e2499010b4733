// Host side of the batched engine: admission by footprint, the step loop,
// the per-system 2BFS transitions and kNN choice, and retirement.
//
// One host thread per engine owns a non-blocking stream.  It enqueues groups
// of steps and, after each group, an asynchronous copy of the per-system
// state into pinned memory; it inspects the copy of group g - 1 while group g
// runs, so the GPU never waits for the host.  Everything the thread decides
// from a copy is enqueued behind the running group; a slot's later copies are
// ignored until they reflect that action (the slot's `guard`).
//
// The 2BFS of the systems that choose eps1 runs on a second stream, beside
// the steps and at its own pace: whenever that stream is idle the thread
// reads its last state copy (BFS fields only), enqueues the transitions it
// calls for (sweep start, next sweep, finish, cancel) and a few BFS rounds,
// then another copy.  Systems whose entries lie within |i - j| <= 31 take
// both sweeps in one launch of one-wave bit-parallel levels on a third
// stream with its own copy, so a long band holds up no one else's rounds.
// After its k0 FP32 iterations a system continues in FP32 until it crosses
// the loosest candidate eps1; there it waits for its features while many
// systems share the steps, or runs ahead copying x~ at each candidate's first
// crossing (batch_runahead: 0 decides by the number of listed systems);
// the state it then restarts from is the one the sequential method stops in,
// so its arithmetic does not depend on that pace.  While any system is being
// admitted or waits for features, groups are shortened to a few ms.

#include "batch_internal.hpp"
#include "knn.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>
#include <vector>

namespace mpcg {
namespace batch {

namespace {

constexpr int kGroupSteps = 8;
// While a system is being admitted or waits for its features, a group lasts
// about this long (the host sees each group's state copy one group later):
// at least two steps, at most the tuned length, a power of two.
constexpr double kGroupLatencyMs = 4.0;
constexpr int kBfsRoundsPerPump = 4;   // BFS rounds enqueued per pass of the BFS stream
constexpr double kEpsClass[8] = {0, 0, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7};

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap).
struct RangeAlloc {
    std::map<int64_t, int64_t> free_;   // start -> length
    void init(int64_t cap)
    {
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    int64_t alloc(int64_t len)
    {
        if (len <= 0) len = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const int64_t s = it->first, rem = it->second - len;
            free_.erase(it);
            if (rem) free_[s + len] = rem;
            return s;
        }
        return -1;
    }
    void release(int64_t s, int64_t len)
    {
        if (len <= 0) len = 1;
        auto nx = free_.lower_bound(s);
        if (nx != free_.end() && nx->first == s + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == s) {
                pv->second += len;
                return;
            }
        }
        free_[s] = len;
    }
};

struct Pending {
    uint64_t id;
    mpcg_request req;
    double t_submit;
};

struct Slot {
    bool used = false;
    uint64_t id = 0;
    mpcg_request req{};
    double t_submit = 0, t_admit = 0, t_feat = 0;
    int32_t slice0 = 0, nslices = 0;
    int64_t entry0 = -1, padded = 0;
    int adm = 0;            // 1: rows and scan enqueued, 2: live
    bool autoe = false;
    int feat = 0;           // 0 not started, 1 sweep 1, 2 sweep 2, 3 finishing, 4 done (or none), 5 cancelling,
                            // 6 band sweeps running (band stream), 7 they gave up: the level kernels next
    bool band_cancel = false;  // cancelled while its band sweeps run: no features once they end
    int split = -1;            // its CG product in two launches: 1 / 0, -1 until a copy shows admission
    bool fall_cc = false;      // feat 7: not connected, start with the components
    bool want_start = false;   // admitted: start the 2BFS on the BFS stream
    bool band = false;         // the 2BFS runs as the one-wave band sweeps (entries within |i - j| <= 31)
    int32_t nh = 0;            // the most offsets of one sign in the band's pattern
    bool fast = false;         // the first sweep runs from vertex 0 without components
    bool want_bfs_cancel = false;
    bool bfs_ready = false;    // pdiam, t, u, ncomp are in f
    int64_t guard = 0;      // ignore state copies of groups before this one
    bool retiring = false;
    int64_t retire_group = 0;
    bool cancel = false;
    int cls = -1;
    int32_t exact = 0;
    double eps1 = 0;
    mpcg_features_t f{};
};

}  // namespace

struct Engine {
    int device = 0;
    mpcg_options opt{};
    const KnnModel *model = nullptr;
    BArena a{};
    hipStream_t s = nullptr;
    BSys *mirror[2] = {nullptr, nullptr};
    int32_t mirror_n[2] = {0, 0};
    int64_t mirror_group[2] = {-1, -1};
    BSys *stage = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // BFS stream: its own state copy (read for the BFS fields only)
    hipStream_t sb = nullptr;
    hipEvent_t evb = nullptr;
    BSys *bmirror = nullptr;
    int32_t bmirror_n = 0;
    // band stream (the one-wave band sweeps) and its state copy
    hipStream_t sband = nullptr;
    hipEvent_t evband = nullptr;
    BSys *bandmirror = nullptr;
    int32_t bandmirror_n = 0;
    bool band_inflight = false;
    bool b_inflight = false;
    std::vector<Slot> slots;
    std::vector<BSys> finals;           // state copy of a slot at completion
    RangeAlloc slices, entries;
    int32_t hi_sys = 0, hi_slice = 0;
    int64_t group = 0;
    // the step's work list: the admitted systems that are not retiring
    bool list_dirty = true;
    int32_t list_slices = 0, list_sys = 0;
    // step groups captured as graphs, by (product grid, per-system grid)
    hipStream_t cap = nullptr;
    std::map<std::tuple<int32_t, int32_t, int32_t, int32_t>, hipGraphExec_t> graphs;   // (grids, steps, dir)
    double step_ms = 0.0;         // recent wall time per step (from the copies' arrival)
    double t_last_copy = 0.0;     // when the previous group's copy was processed
    int len_k[2] = {0, 0};        // steps of the group of each copy slot
    bool graphs_ok = true;
    // scheduling knobs: mpcg_tuning's batch_* fields
    int small_levels = kSmallBfsLevels;
    int small_cap = kSmallBfsCapDefault;
    int64_t small_work = INT64_MAX;   // frontier x lane slots after which a one-block launch stops: no limit
    int bfs_rounds = kBfsRoundsPerPump;
    int level_grid = 1024;
    int group_steps = kGroupSteps;
    bool band_on = true;   // batch_bfs_band

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> pending;        // guarded by mu
    std::deque<std::pair<uint64_t, mpcg_stats>> done;   // guarded by mu
    std::vector<uint64_t> cancels;      // guarded by mu
    int32_t n_queued = 0, n_active = 0; // guarded by mu
    bool stop = false;                  // guarded by mu
    std::atomic<bool> failed{false};
    uint64_t next_id = 1;               // guarded by mu
    std::thread th;

    std::deque<Pending> local;          // taken from `pending` by the thread

    void run();
    bool step_once();
    bool rebuild_list();
    bool launch_group(int len);
    bool dir_needed() const;
    bool band_pump();
    void process_band(const BSys *m, int32_t cnt);
    int group_len() const;
    void drop_graphs();
    void finish(Slot &sl, const BSys *M, int status_override);
    void recompute_hi();
    void admit();
    void process(const BSys *m, int32_t cnt, int64_t gi);
    void process_slots(const BSys *m, int32_t cnt, int64_t gi, AdmitList &l2);
    bool bfs_pump();
    bool process_bfs(const BSys *m, int32_t cnt);
    void fail_all(int status);
};

void Engine::recompute_hi()
{
    int32_t hs = 0, hl = 0;
    for (int32_t i = 0; i < (int32_t)slots.size(); ++i) {
        if (!slots[i].used) continue;
        hs = i + 1;
        if (slots[i].slice0 + slots[i].nslices > hl) hl = slots[i].slice0 + slots[i].nslices;
    }
    hi_sys = hs;
    hi_slice = hl;
}

void Engine::finish(Slot &sl, const BSys *M, int status_override)
{
    mpcg_stats st{};
    st.eps1_class = sl.cls;
    st.eps1_used = sl.req.eps1 == MPCG_EPS1_NONE ? -1.0 : (sl.autoe ? sl.eps1 : sl.req.eps1);
    if (M) {
        st.n1 = M->n1;
        st.n2 = M->n2;
        st.restarts = M->restarts;
        st.flags = M->flags | (sl.exact ? MPCG_FLAG_KNN_EXACT : 0);
        st.status = M->status;
        st.relres_sp = M->relres_sp;
        st.relres_restart_true = M->relres_restart;
        st.relres_final_true = M->relres_final;
    }
    if (status_override) st.status = status_override;
    st.I_third = st.n1 / 3.0 + st.n2;
    st.t_total_ms = now_ms() - sl.t_submit;
    st.t_feat_ms = sl.t_feat > 0 ? sl.t_feat - sl.t_admit : 0.0;
    st.feat = sl.f;
    std::lock_guard<std::mutex> lk(mu);
    done.emplace_back(sl.id, st);
    n_active -= 1;
}

void Engine::fail_all(int status)
{
    failed = true;
    for (auto &sl : slots) {
        if (!sl.used) continue;
        finish(sl, nullptr, status);
        sl.used = false;
    }
    std::lock_guard<std::mutex> lk(mu);
    for (auto &p : local) {
        mpcg_stats st{};
        st.status = status;
        done.emplace_back(p.id, st);
    }
    for (auto &p : pending) {
        mpcg_stats st{};
        st.status = status;
        done.emplace_back(p.id, st);
    }
    n_queued = 0;
    local.clear();
    pending.clear();
}

// Admission, stage 1: a free slot and slice range; rows and the padded-entry
// scan are enqueued (stage 2 runs once a state copy shows the scan's total).
void Engine::admit()
{
    // the systems admitted now share one launch per kernel of stage 1, and
    // consecutive slots' staged states one copy
    AdmitList l{};
    int32_t run0 = 0, runn = 0;
    auto flush_copy = [&]() {
        if (runn > 0 && hipMemcpyAsync(&a.sys[run0], &stage[run0], sizeof(BSys) * (size_t)runn,
                                       hipMemcpyHostToDevice, s) != hipSuccess)
            failed = true;
        runn = 0;
    };
    auto flush = [&]() {
        flush_copy();
        if (!failed) launch_admit_stage1(s, a, l);
        l = AdmitList{};
    };
    while (!local.empty() && !failed) {
        int32_t slot = -1;
        for (int32_t i = 0; i < (int32_t)slots.size(); ++i)
            if (!slots[i].used) { slot = i; break; }
        if (slot < 0) break;
        Pending p = local.front();
        const mpcg_request &r = p.req;
        const int32_t n = (int32_t)r.A.n;
        const int32_t nsl = (n + 63) / 64;
        const int64_t s0 = slices.alloc(nsl);
        if (s0 < 0) break;   // wait for space
        local.pop_front();
        Slot &sl = slots[slot];
        sl = Slot{};
        sl.used = true;
        sl.id = p.id;
        sl.req = r;
        sl.t_submit = p.t_submit;
        sl.t_admit = now_ms();
        sl.slice0 = (int32_t)s0;
        sl.nslices = nsl;
        sl.adm = 1;
        sl.autoe = r.eps1 == MPCG_EPS1_AUTO;
        sl.guard = group;   // the copy after the group enqueued next holds the scan
        sl.f.n = r.A.n;
        sl.f.m = r.A.nnz;
        BSys &S = stage[slot];
        std::memset(&S, 0, sizeof(BSys));
        S.row0 = (int32_t)s0 * 64;
        S.n = n;
        S.slice0 = (int32_t)s0;
        S.nslices = nsl;
        S.nnz = r.A.nnz;
        S.auto_eps = sl.autoe ? 1 : 0;
        S.k0 = opt.k0 > 0 ? opt.k0 : 20;
        S.tol_abs = opt.tol_mode == 1;
        S.max_restarts = opt.max_restarts >= 0 ? opt.max_restarts : 5;
        const int64_t mi1 = opt.maxit1 > 0 ? opt.maxit1 : n;
        const int64_t mi2 = opt.maxit2 > 0 ? opt.maxit2 : (10 * (int64_t)n > 1000 ? 10 * (int64_t)n : 1000);
        S.maxit1 = (int32_t)(mi1 < 0x7ffffff0 ? mi1 : 0x7ffffff0);
        S.maxit2 = (int32_t)(mi2 < 0x7ffffff0 ? mi2 : 0x7ffffff0);
        const int64_t avg = (r.A.nnz + n - 1) / n;
        int lanes = 1;
        while (lanes < avg && lanes < 32) lanes <<= 1;
        S.lanes = lanes;
        S.eps2 = r.eps2;
        S.mode = kFree;
        if (runn > 0 && slot == run0 + runn) {
            ++runn;
        } else {
            flush_copy();
            run0 = slot;
            runn = 1;
        }
        const int k = l.cnt++;
        l.sys[k] = slot;
        l.nsl[k] = nsl;
        l.rp[k] = r.A.row_ptr;
        l.rp_i64[k] = r.A.row_ptr_is_i64;
        l.b[k] = r.b;
        if (l.cnt == kAdmitList) flush();
        {
            std::lock_guard<std::mutex> lk(mu);
            n_queued -= 1;
            n_active += 1;
        }
        recompute_hi();
    }
    if (l.cnt > 0 || runn > 0) flush();
}

void Engine::process(const BSys *m, int32_t cnt, int64_t gi)
{
    AdmitList l2{};   // stage 2 of the systems whose scan this copy shows: one launch per kernel
    process_slots(m, cnt, gi, l2);
    if (!failed) launch_admit_stage2(s, a, l2);
}

void Engine::process_slots(const BSys *m, int32_t cnt, int64_t gi, AdmitList &l2)
{
    for (int32_t i = 0; i < (int32_t)slots.size() && i < cnt; ++i) {
        Slot &sl = slots[i];
        if (!sl.used || gi < sl.guard) continue;
        const BSys &M = m[i];
        if (sl.adm == 1) {
            sl.padded = M.padded;
            const int64_t e0 = entries.alloc(sl.padded);
            if (e0 < 0) {
                if (sl.padded > a.max_entries) {
                    finish(sl, nullptr, MPCG_ENOMEM);
                } else {   // back to the queue until entries free up
                    std::lock_guard<std::mutex> lk(mu);
                    local.push_front(Pending{sl.id, sl.req, sl.t_submit});
                    n_queued += 1;
                    n_active -= 1;
                }
                launch_release(s, a, i, sl.slice0, sl.nslices);
                slices.release(sl.slice0, sl.nslices);
                sl.used = false;
                recompute_hi();
                continue;
            }
            sl.entry0 = e0;
            stage[i].entry0 = e0;
            const int k = l2.cnt++;
            l2.sys[k] = i;
            l2.nsl[k] = sl.nslices;
            l2.rp[k] = sl.req.A.row_ptr;
            l2.rp_i64[k] = sl.req.A.row_ptr_is_i64;
            l2.col[k] = sl.req.A.col_idx;
            l2.val[k] = sl.req.A.val;
            l2.eps1[k] = sl.req.eps1;
            l2.entry0[k] = e0;
            if (l2.cnt == kAdmitList) {
                launch_admit_stage2(s, a, l2);
                l2 = AdmitList{};
            }
            sl.adm = 2;
            sl.guard = group + 1;
            list_dirty = true;
            continue;
        }
        if (sl.split < 0) sl.split = M.split;   // this copy follows the admission (guard)
        if (sl.retiring) {
            if (gi >= sl.retire_group) {
                finish(sl, &finals[i], 0);
                launch_release(s, a, i, sl.slice0, sl.nslices);
                slices.release(sl.slice0, sl.nslices);
                entries.release(sl.entry0, sl.padded);
                sl.used = false;
                recompute_hi();
            }
            continue;
        }
        if (sl.cancel) {
            launch_cancel(s, a, i);
            sl.cancel = false;
            if (sl.autoe && sl.feat == 6) sl.band_cancel = true;   // feat 4 once the band sweeps have ended
            else if (sl.autoe && sl.feat >= 1 && sl.feat <= 3) sl.want_bfs_cancel = true;   // feat 5, then 4
            else if (sl.feat != 5) sl.feat = 4;   // 5: a BFS cancel is already under way
            sl.want_start = false;
            sl.guard = group + 1;
            continue;
        }
        if (sl.autoe && sl.feat < 4) {
            if (sl.feat == 0 && !sl.want_start) {
                if (M.err || M.mode == kDone) {
                    sl.feat = 4;   // malformed input or nothing to solve: no features
                } else {
                    sl.want_start = true;
                    sl.band = band_on && M.bw <= kBandMaxBw;
                    sl.nh = std::max(__builtin_popcountll(M.doffs & 0xffffffffull), __builtin_popcountll(M.doffs >> 33));
                }
            } else if (sl.feat == 3 && sl.bfs_ready && !(M.mode == kCg32 && M.k0_used == 0)) {
                sl.f.k0_used = M.k0_used;
                double sum = 0.0;
                for (int j = 0; j < M.k0_used && j < kK0Max; ++j) sum = sum + M.ratios[j];
                sl.f.v = M.k0_used > 0 ? sum / (double)M.k0_used : 0.0;
                const double chi[4] = {(double)sl.f.n, (double)sl.f.m, (double)sl.f.pdiam, sl.f.v};
                sl.exact = 0;
                const int cls = knn_select(*model, chi, opt.knn_k, &sl.exact);
                sl.cls = (cls >= 2 && cls <= 7) ? cls : 4;
                sl.eps1 = kEpsClass[sl.cls];
                launch_set_eps(s, a, i, sl.eps1, sl.cls - 2);
                sl.t_feat = now_ms();
                sl.feat = 4;
                sl.guard = group + 1;
                continue;
            }
        }
        if (M.mode == kDone && (!sl.autoe || sl.feat == 4)) {
            const int st = M.status;
            if (st != MPCG_EINVAL && st != MPCG_ECANCELED && sl.req.x) {
                if (hipMemcpyAsync(sl.req.x, a.x64 + M.row0, sizeof(double) * (size_t)M.n, hipMemcpyDeviceToDevice,
                                   s) != hipSuccess) {
                    failed = true;
                    return;
                }
            }
            // the statistics are final in this copy; x is complete once the state copy of
            // the next group has been taken (same stream)
            finals[i] = M;
            sl.retiring = true;
            sl.retire_group = group + 1;
            sl.guard = group + 1;
            list_dirty = true;
        }
    }
}

// BFS transitions from the BFS stream's state copy (that stream is idle).
bool Engine::process_bfs(const BSys *m, int32_t cnt)
{
    bool enq = false;
    for (int32_t i = 0; i < (int32_t)slots.size() && i < cnt; ++i) {
        Slot &sl = slots[i];
        if (!sl.used || !sl.autoe) continue;
        const BSys &M = m[i];
        if (sl.feat == 5) {   // the BFS cancel ran before this copy
            sl.feat = 4;
            continue;
        }
        if (sl.feat < 1 || sl.feat > 3) continue;
        if (M.bfs_err & kErrGuard) {   // a bounded loop ran out: no features, the solve is cancelled
            launch_cancel(s, a, i);
            sl.guard = group + 1;
            launch_bfs_cancel(sb, a, i);
            sl.feat = 5;
            enq = true;
            continue;
        }
        if (sl.feat == 1 && M.bfs_mode == kBfsSwept) {
            launch_bfs_next_sweep(sb, a, i, (int32_t)sl.f.n);
            sl.feat = 2;
            enq = true;
        } else if (sl.feat == 2 && M.bfs_mode == kBfsSwept) {
            if (sl.fast && M.reached < (int32_t)sl.f.n) {
                // not connected: start over with the connected components
                launch_bfs_start(sb, a, i, (int32_t)sl.f.n);
                sl.fast = false;
                sl.feat = 1;
            } else {
                launch_bfs_finish(sb, a, i, (int32_t)sl.f.n);
                sl.feat = 3;
            }
            enq = true;
        } else if (sl.feat == 3 && M.bfs_mode == kBfsDone && !sl.bfs_ready) {
            sl.f.pdiam = M.pdiam;
            sl.f.bfs_t = M.bfs_t;
            sl.f.bfs_u = M.bfs_u;
            sl.f.n_components = M.ncomp;
            sl.bfs_ready = true;
        }
    }
    return enq;
}

// Results of the band stream's last launch (its own state copy, read for the
// band systems' BFS fields only).
void Engine::process_band(const BSys *m, int32_t cnt)
{
    for (int32_t i = 0; i < (int32_t)slots.size() && i < cnt; ++i) {
        Slot &sl = slots[i];
        if (!sl.used || sl.feat != 6) continue;
        const BSys &M = m[i];
        if (sl.band_cancel) {
            sl.feat = 4;
        } else if (M.bfs_mode == kBfsDone) {
            sl.f.pdiam = M.pdiam;
            sl.f.bfs_t = M.bfs_t;
            sl.f.bfs_u = M.bfs_u;
            sl.f.n_components = M.ncomp;
            sl.bfs_ready = true;
            sl.feat = 3;
        } else {   // not connected (the components first), or a frontier too wide for the window
            sl.fall_cc = M.band_fail == 2;
            sl.feat = 7;
        }
    }
}

// The band stream, when idle: the systems waiting for band sweeps, grouped
// by offset count (a launch unrolls its level for the most offsets its
// systems have), then a state copy.  Runs beside the BFS stream, so a long
// band does not hold up the level kernels' rounds.
bool Engine::band_pump()
{
    if (band_inflight) {
        const hipError_t q = hipEventQuery(evband);
        if (q == hipErrorNotReady) return true;
        if (q != hipSuccess) return false;
        band_inflight = false;
        process_band(bandmirror, bandmirror_n);
    }
    BandList bl[4] = {};
    bool any = false;
    for (int32_t i = 0; i < (int32_t)slots.size(); ++i) {
        Slot &sl = slots[i];
        if (!sl.used || !sl.autoe || !sl.want_start || !sl.band) continue;
        launch_band_masks(sband, a, i, sl.nslices);
        const int c = sl.nh <= 4 ? 0 : sl.nh <= 8 ? 1 : sl.nh <= 16 ? 2 : 3;
        BandList &l = bl[c];
        l.slot[l.cnt++] = i;
        l.nh_max = std::max(l.nh_max, sl.nh);
        if (l.cnt == kBandList) {
            launch_bfs_band(sband, a, l);
            l = BandList{};
        }
        sl.want_start = false;
        sl.feat = 6;
        any = true;
    }
    if (!any) return true;
    for (const BandList &l : bl) launch_bfs_band(sband, a, l);   // nothing for an empty list
    if (hipGetLastError() != hipSuccess) return false;
    bandmirror_n = hi_sys;
    if (hipMemcpyAsync(bandmirror, a.sys, sizeof(BSys) * (size_t)hi_sys, hipMemcpyDeviceToHost, sband) !=
            hipSuccess ||
        hipEventRecord(evband, sband) != hipSuccess)
        return false;
    band_inflight = true;
    return true;
}

// One pass of the BFS stream, if it is idle: its last copy is processed,
// then transitions, rounds and the next copy are enqueued.  Never blocks.
bool Engine::bfs_pump()
{
    if (!band_pump()) return false;
    if (b_inflight) {
        const hipError_t q = hipEventQuery(evb);
        if (q == hipErrorNotReady) return true;
        if (q != hipSuccess) return false;
        b_inflight = false;
    }
    // transitions enqueued from the copy need a copy behind them
    bool enq = !b_inflight && bmirror_n > 0 ? process_bfs(bmirror, bmirror_n) : false;
    bool run = false;
    for (int32_t i = 0; i < (int32_t)slots.size(); ++i) {
        Slot &sl = slots[i];
        if (!sl.used || !sl.autoe) continue;
        if (sl.want_bfs_cancel) {
            launch_bfs_cancel(sb, a, i);
            sl.want_bfs_cancel = false;
            sl.feat = 5;
            enq = true;
        }
        if (sl.want_start && !sl.band) {
            launch_bfs_fast_start(sb, a, i, (int32_t)sl.f.n);
            sl.fast = true;
            sl.want_start = false;
            sl.feat = 1;
            enq = true;
        }
        if (sl.feat == 7) {   // the band sweeps gave up: the level kernels
            if (sl.fall_cc) launch_bfs_start(sb, a, i, (int32_t)sl.f.n);
            else launch_bfs_fast_start(sb, a, i, (int32_t)sl.f.n);
            sl.fast = !sl.fall_cc;
            sl.feat = 1;
            enq = true;
        }
        if (sl.feat == 1 || sl.feat == 2) run = true;
        if ((sl.feat == 3 && !sl.bfs_ready) || sl.feat == 5) enq = true;   // waiting for a copy that shows the result
    }
    if (run)
        for (int r = 0; r < bfs_rounds; ++r) launch_bfs_round(sb, a, hi_sys, small_levels, small_cap, small_work, level_grid);
    if (hipGetLastError() != hipSuccess) return false;
    if (!(enq || run) || hi_sys <= 0) return true;
    bmirror_n = hi_sys;
    if (hipMemcpyAsync(bmirror, a.sys, sizeof(BSys) * (size_t)hi_sys, hipMemcpyDeviceToHost, sb) != hipSuccess ||
        hipEventRecord(evb, sb) != hipSuccess)
        return false;
    b_inflight = true;
    return true;
}

// Grid sizes of the step's launches, rounded up to m * 2^e with 8 <= m < 16
// (at most one block in eight past the listed work) so that few distinct
// sizes -- and captured graphs -- occur.
static int32_t coarse_grid(int64_t x)
{
    if (x <= 16) return (int32_t)(x > 0 ? x : 1);
    int e = 0;
    while ((x >> e) >= 16) ++e;
    int64_t m = x >> e;
    if ((m << e) < x) ++m;
    return (int32_t)(m << e);
}

// The work list: systems whose rows and entries are in place and that have
// not been seen to finish, in slot order.
bool Engine::rebuild_list()
{
    ListChunk c{};
    int32_t total = 0, nsys = 0;
    std::vector<int32_t> ids;
    for (int32_t i = 0; i < (int32_t)slots.size(); ++i)
        if (slots[i].used && slots[i].adm == 2 && !slots[i].retiring) ids.push_back(i);
    for (int32_t i : ids) total += slots[i].nslices;
    nsys = (int32_t)ids.size();
    int32_t pre = 0;
    size_t k = 0;
    do {
        c.first = (int32_t)k;
        c.n = 0;
        for (; k < ids.size() && c.n < kListChunk; ++k, ++c.n) {
            const Slot &sl = slots[ids[k]];
            c.slot[c.n] = ids[k];
            c.slice0[c.n] = sl.slice0;
            c.nslices[c.n] = sl.nslices;
            c.pre[c.n] = pre;
            pre += sl.nslices;
        }
        c.last = k == ids.size() ? 1 : 0;
        c.total_slices = total;
        c.total_sys = nsys;
        launch_worklist(s, a, c);
    } while (k < ids.size());
    if (hipGetLastError() != hipSuccess) return false;
    list_slices = total;
    list_sys = nsys;
    list_dirty = false;
    return true;
}

void Engine::drop_graphs()
{
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
}

// One group of steps: a graph replay when the group is captured (once per
// pair of grid sizes), else plain launches.
bool Engine::launch_group(int len)
{
    const int32_t gsl = coarse_grid((list_slices + kSlicesPerBlock - 1) / kSlicesPerBlock);
    const int32_t gsys = coarse_grid(list_sys);
    if (graphs_ok) {
        const bool dir = dir_needed();
        const auto key = std::make_tuple(gsl, gsys, (int32_t)len, (int32_t)dir);
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            if (graphs.size() >= 64) drop_graphs();
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                for (int j = 0; j < len; ++j) launch_step(cap, a, gsl, gsys, dir);
                ok = hipStreamEndCapture(cap, &g) == hipSuccess && g != nullptr;
            }
            ok = ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            if (!ok) {
                graphs_ok = false;   // plain launches from now on
            } else {
                it = graphs.emplace(key, ex).first;
            }
        }
        if (graphs_ok) return hipGraphLaunch(it->second, s) == hipSuccess;
    }
    const bool dir = dir_needed();
    for (int j = 0; j < len; ++j) launch_step(s, a, gsl, gsys, dir);
    return hipGetLastError() == hipSuccess;
}

// Some listed system may gather a stored direction: its split flag is set on
// the device at admission and reaches the host one copy later, so a system
// not yet seen counts as split.
bool Engine::dir_needed() const
{
    for (const auto &sl : slots)
        if (sl.used && !sl.retiring && sl.adm == 2 && sl.split != 0) return true;
    return false;
}

// Steps of the next group: the tuned length, or shorter while a system is
// being admitted or waits for its features (their latency is counted in
// groups).
int Engine::group_len() const
{
    bool waiting = false;
    for (const auto &sl : slots)
        if (sl.used && !sl.retiring && (sl.adm == 1 || (sl.autoe && sl.feat < 4))) waiting = true;
    if (!waiting || step_ms <= 0.0) return group_steps;
    int want = (int)(kGroupLatencyMs / step_ms);
    int len = 2;
    while (len * 2 <= want && len * 2 <= group_steps) len *= 2;
    return len < group_steps ? len : group_steps;
}

bool Engine::step_once()
{
    // new submissions and cancellations
    {
        std::lock_guard<std::mutex> lk(mu);
        while (!pending.empty()) {
            local.push_back(pending.front());
            pending.pop_front();
        }
        for (uint64_t id : cancels) {
            bool found = false;
            for (auto it = local.begin(); it != local.end(); ++it) {
                if (it->id != id) continue;
                mpcg_stats st{};
                st.status = MPCG_ECANCELED;
                done.emplace_back(id, st);
                local.erase(it);
                n_queued -= 1;
                found = true;
                break;
            }
            if (found) continue;
            for (auto &sl : slots)
                if (sl.used && sl.id == id && !sl.retiring) sl.cancel = true;
        }
        cancels.clear();
    }
    admit();
    if (failed) return false;
    bool any_used = false, any_live = false;
    for (auto &sl : slots) {
        if (!sl.used) continue;
        any_used = true;
        if (sl.adm == 2 && !sl.retiring) any_live = true;
    }
    if (!any_used) return true;
    if (!bfs_pump()) return false;
    const int k = (int)(group & 1);
    if (list_dirty && !rebuild_list()) return false;
    const int len = group_len();
    len_k[k] = any_live && list_sys > 0 ? len : 0;
    if (any_live && list_sys > 0 && !launch_group(len)) return false;
    if (hipGetLastError() != hipSuccess) return false;
    mirror_n[k] = hi_sys;
    mirror_group[k] = group;
    if (hi_sys > 0 &&
        hipMemcpyAsync(mirror[k], a.sys, sizeof(BSys) * (size_t)hi_sys, hipMemcpyDeviceToHost, s) != hipSuccess)
        return false;
    if (hipEventRecord(ev[k], s) != hipSuccess) return false;
    const int kp = k ^ 1;
    if (mirror_group[kp] >= 0 && mirror_group[kp] == group - 1) {
        // wait for the previous group's copy, keeping the BFS stream fed meanwhile
        for (;;) {
            const hipError_t q = hipEventQuery(ev[kp]);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return false;
            if (!bfs_pump()) return false;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        // the previous group ran since the copy before it was processed
        const double t = now_ms();
        if (t_last_copy > 0.0 && len_k[kp] > 0) step_ms = (t - t_last_copy) / len_k[kp];
        t_last_copy = t;
        process(mirror[kp], mirror_n[kp], group - 1);
        if (failed) return false;
    }
    group += 1;
    return true;
}

void Engine::run()
{
    if (hipSetDevice(device) != hipSuccess) {
        fail_all(MPCG_EDEVICE);
        return;
    }
    for (;;) {
        bool idle;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            bool any_used = false;
            for (auto &sl : slots) any_used = any_used || sl.used;
            idle = !any_used && local.empty() && pending.empty() && cancels.empty();
            if (idle) {
                cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        if (!step_once()) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamSynchronize(sb);
            (void)hipStreamSynchronize(sband);
            fail_all(MPCG_EDEVICE);
            std::unique_lock<std::mutex> lk(mu);
            while (!stop) cv.wait_for(lk, std::chrono::milliseconds(20));
            break;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(sb);
    (void)hipStreamSynchronize(sband);
}

// ------------------------------------------------------------ interface --

Engine *engine_create(int device, const mpcg_options &opt, const mpcg_tuning &tune, const KnnModel *model,
                      void *arena, size_t bytes,
                      int64_t max_rows, int64_t max_entries, int32_t max_sys, int *status)
{
    const int64_t max_slices = (max_rows + 63) / 64;
    if (max_slices <= 0 || max_slices > (0x7fffffff / 64) || max_entries <= 0 || max_sys <= 0 ||
        max_sys > (1 << 16) || !arena) {
        *status = MPCG_EINVAL;
        return nullptr;
    }
    if (bytes < arena_bytes(max_sys, (int32_t)max_slices, max_entries)) {
        *status = MPCG_ENOMEM;
        return nullptr;
    }
    Engine *e = new (std::nothrow) Engine();
    if (!e) {
        *status = MPCG_EDEVICE;
        return nullptr;
    }
    e->device = device;
    e->opt = opt;
    e->small_levels = tune.batch_small_levels;
    e->small_cap = tune.batch_small_cap;
    e->bfs_rounds = tune.batch_bfs_rounds;
    e->level_grid = tune.batch_level_grid;
    e->group_steps = tune.batch_group_steps;
    e->model = model;
    e->a = carve(arena, max_sys, (int32_t)max_slices, max_entries);
    e->a.acc32 = opt.dot_acc;
    // nontemporal matrix loads where the arena's FP64 matrices (8-byte values,
    // 4-byte columns) can exceed the Infinity Cache, unless the tuning says
    e->a.nt = tune.sell_stream < 0 ? (max_entries * 12 > kInfinityCacheBytes ? 1 : 0) : tune.sell_stream;
    // 0: wait when more than kHoldAboveSystems systems are listed; 1: always
    // run ahead; 2: always wait
    e->a.hold_above = tune.batch_runahead == 1 ? INT32_MAX : tune.batch_runahead == 2 ? -1 : kHoldAboveSystems;
    e->band_on = tune.batch_bfs_band != 0;
    e->slots.resize(max_sys);
    e->finals.resize(max_sys);
    e->slices.init(max_slices);
    e->entries.init(max_entries);
    bool ok = hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&e->sb, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&e->sband, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&e->evband, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void **)&e->bandmirror, sizeof(BSys) * (size_t)max_sys, hipHostMallocDefault) ==
                  hipSuccess &&
              hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&e->evb, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void **)&e->bmirror, sizeof(BSys) * (size_t)max_sys, hipHostMallocDefault) ==
                  hipSuccess;
    for (int k = 0; k < 2 && ok; ++k) {
        ok = hipHostMalloc((void **)&e->mirror[k], sizeof(BSys) * (size_t)max_sys, hipHostMallocDefault) ==
                 hipSuccess &&
             hipEventCreateWithFlags(&e->ev[k], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipHostMalloc((void **)&e->stage, sizeof(BSys) * (size_t)max_sys, hipHostMallocDefault) == hipSuccess;
    if (ok) {
        ok = hipMemsetAsync(e->a.sys, 0, sizeof(BSys) * (size_t)max_sys, e->s) == hipSuccess;
        launch_fill_slices(e->s, e->a);
        ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(e->s) == hipSuccess;
    }
    if (!ok) {
        engine_destroy(e);
        *status = MPCG_EDEVICE;
        return nullptr;
    }
    e->th = std::thread([e]() { e->run(); });
    *status = MPCG_OK;
    return e;
}

void engine_destroy(Engine *e)
{
    if (!e) return;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
    }
    e->cv.notify_all();
    if (e->th.joinable()) e->th.join();
    if (e->s) {
        (void)hipStreamSynchronize(e->s);
        (void)hipStreamDestroy(e->s);
    }
    if (e->sb) {
        (void)hipStreamSynchronize(e->sb);
        (void)hipStreamDestroy(e->sb);
    }
    if (e->sband) {
        (void)hipStreamSynchronize(e->sband);
        (void)hipStreamDestroy(e->sband);
    }
    if (e->evband) (void)hipEventDestroy(e->evband);
    if (e->bandmirror) (void)hipHostFree(e->bandmirror);
    e->drop_graphs();
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->evb) (void)hipEventDestroy(e->evb);
    if (e->bmirror) (void)hipHostFree(e->bmirror);
    for (auto &v : e->ev) if (v) (void)hipEventDestroy(v);
    for (auto &m : e->mirror) if (m) (void)hipHostFree(m);
    if (e->stage) (void)hipHostFree(e->stage);
    delete e;
}

int engine_submit(Engine *e, const mpcg_request *reqs, int32_t count, uint64_t *ids)
{
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->failed) return MPCG_EDEVICE;
    const double t = now_ms();
    for (int32_t i = 0; i < count; ++i) {
        const uint64_t id = e->next_id++;
        ids[i] = id;
        e->pending.push_back(Pending{id, reqs[i], t});
        e->n_queued += 1;
    }
    e->cv.notify_one();
    return MPCG_OK;
}

int engine_poll(Engine *e, uint64_t *ids, mpcg_stats *stats, int32_t cap, int32_t *n_done)
{
    std::lock_guard<std::mutex> lk(e->mu);
    int32_t k = 0;
    while (k < cap && !e->done.empty()) {
        ids[k] = e->done.front().first;
        if (stats) stats[k] = e->done.front().second;
        e->done.pop_front();
        ++k;
    }
    *n_done = k;
    return MPCG_OK;
}

int engine_cancel(Engine *e, uint64_t id)
{
    std::lock_guard<std::mutex> lk(e->mu);
    if (id == 0 || id >= e->next_id) return MPCG_EINVAL;
    e->cancels.push_back(id);
    e->cv.notify_one();
    return MPCG_OK;
}

int engine_load(Engine *e, int32_t *queued, int32_t *active)
{
    std::lock_guard<std::mutex> lk(e->mu);
    if (queued) *queued = e->n_queued;
    if (active) *active = e->n_active;
    return MPCG_OK;
}

int64_t engine_max_slices(const Engine *e) { return e->a.max_slices; }
int64_t engine_max_entries(const Engine *e) { return e->a.max_entries; }

}  // namespace batch
}  // namespace mpcg
