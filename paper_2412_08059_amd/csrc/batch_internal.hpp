// Batched engine: many independent systems solved together.
//
// Every admitted system owns a contiguous range of 64-row slices in one
// shared row space (its rows padded to a multiple of 64, so a slice never
// holds rows of two systems) and a contiguous range of SELL-64 entries.  The
// union of the systems is a block-diagonal matrix; one "step" advances every
// system by one unit of its own state machine with a fixed set of launches
// that cover all slices at once:
//
//   k_b_product   per slice: the CG product, the restart residual or the
//                 final-check residual of the slice's system, as its mode says;
//                 one partial per slice
//   k_b_scalar1   one block per system: its partials -> delta / alpha, or the
//                 restart and final-check decisions
//   k_b_update    per slice: r -= alpha q, x += alpha d, partial of r.r
//   k_b_scalar2   one block per system: gamma, stop tests, beta, v ratios
//   k_b_bfs_*     2BFS levels of the systems whose features are pending, on a
//                 stream of their own beside the steps
//
// Per-system sums are taken over that system's slice partials in a fixed
// order, so a system's arithmetic does not depend on which other systems
// share the batch: a solve gives the same bits alone and in any mix.

#pragma once

#include "knn.hpp"
#include "mpcg_internal.hpp"

namespace mpcg {
namespace batch {

enum Mode : int32_t {
    kFree = 0,      // slot unused
    kHold = 1,      // FP32 prefix done, waiting for eps1 (Algorithm II)
    kCg32 = 2,
    kRestart = 3,   // next product forms r = b - A x in FP64
    kCg64 = 4,
    kResid = 5,     // next product forms ||b - A x||
    kDone = 6,
};

enum RestartSrc : int32_t { kSrcX32 = 0, kSrcX64 = 1, kSrcZero = 2, kSrcSnap = 3 };

// Why a system's FP32 run-ahead stopped before its eps1 was known (kRaWait:
// the engine holds systems after their k0 prefix until eps1 is known).
enum RunAheadStop : int32_t { kRaNone = 0, kRaBreakdown = 1, kRaMaxit = 2, kRaAllCrossed = 3, kRaWait = 4 };

enum BfsMode : int32_t {
    kBfsNone = 0,
    kBfsRun = 1,    // a sweep is expanding
    kBfsSwept = 2,  // a sweep ended; the host finishes it (argmax, next seed)
    kBfsDone = 3,   // pdiam, t, u, ncomp are final
};

constexpr int kSlicesPerBlock = kBlock / 64;
constexpr int32_t kErrGuard = 64;     // a bounded device loop ran out (union-find)
constexpr int kSmallBfsCap = 2048;   // frontier kept in LDS by the one-block-per-system kernel
constexpr int kSmallBfsCapDefault = 512;   // default of the largest frontier that kernel takes (<= kSmallBfsCap)
constexpr int kVisBits = 1 << 20;     // rows up to which that kernel keeps the visited set in LDS (128 KB)
constexpr int kSmallBfsLevels = 64;  // default of the levels one launch may expand for one system

struct alignas(256) BSys {
    // set at admission
    int32_t row0, n, slice0, nslices;
    int64_t nnz, entry0;
    int32_t auto_eps, k0, tol_abs, max_restarts;
    int32_t maxit1, maxit2, lanes, err;
    double eps2;
    // recurrence
    int32_t mode, ph_it, n1, n2;
    int32_t restarts, flags, status, src;
    int32_t upd, k0_used, eps_set, pend;   // pend: status to report after the final residual
    double gamma, gamma_prev, delta, alpha, beta, bb, thr1, thr2;
    double relres_sp, relres_restart, relres_final;
    double ratios[kK0Max];
    // Algorithm II run-ahead: after the k0 prefix, until eps1 is set, the FP32
    // recurrence continues and x~ is copied at the first crossing of each
    // candidate eps1 (copy taken by the next product, snap_mask: classes due)
    double spec_thr[kNumEps];
    double cross_gamma[kNumEps];
    int32_t cross_iter[kNumEps];
    int32_t snap_mask, snap_ci, ra_stop;
    int32_t spec;                          // the FP64 phase runs speculatively from the tightest candidate
    // 2BFS
    int32_t bfs_mode, bfs_sweep, bfs_level, bfs_cnt;
    int32_t bfs_nxt, ncomp, pdiam, bfs_t;
    int32_t bfs_u, small, bfs_err;         // bfs_err: kErrGuard from the BFS kernels
    int32_t vis_lvl;                       // BArena::vis of the system matches dist after this level
    int32_t reached;                       // vertices the first sweep reached (counted at its end)
    int32_t bw;                            // max |i - j| over the entries (admission)
    unsigned long long doffs;              // bit d + 32: some entry at j - i = d, 0 < |d| <= 31 (admission)
    int32_t band_fail;                     // band 2BFS: 1 frontier too wide for its window, 2 not connected
    int32_t split;                         // CG product in two launches (scattered columns, set at admission)
    int64_t padded;                        // SELL-64 entries of the system (admission scan)
    unsigned long long comp_best;
    int64_t item0;                         // first BFS work item of this system in the current level
};

// Device pointers of the batch arena.
struct BArena {
    BSys *sys;
    int32_t max_sys, max_slices;
    int64_t max_entries;
    // per slice
    int32_t *slice_w, *sys_of_slice;
    int64_t *slice_off;                    // local to the system's entry range
    double *pslice;                        // 2 per slice
    // per row
    int32_t *rowlen;
    double *b64, *x64, *r64, *q64, *dA64, *dB64;
    float *x32, *r32, *q32, *dA32, *dB32;
    float *snap32;                         // kNumEps copies of x~, copy t at t * max_slices * 64
    int32_t *dist, *q0, *q1, *label, *tarr;
    uint32_t *vis;                         // visited bits of the small-level BFS and of the band sweeps, one per row
    uint32_t *dm;                          // band 2BFS: per 32-row word w of the row space, 64 words
                                           // dm[w * 64 + d + 32], bit b: row 32 w + b is reached from
                                           // row 32 w + b - d (an entry at offset d of that row)
    unsigned long long *best;
    // per entry
    int32_t *col;
    double *v64;
    float *v32;
    // BFS work lists
    int32_t *act_sys;                      // systems expanding a large level this step
    int64_t *act_pre;                      // their exclusive item prefix
    int32_t *small_sys;                    // systems expanding small levels this step
    int32_t *counts;                       // [0] = #act, [1] = #small, [2] = admission error (unused)
    int64_t *items;                        // total items of the large level
    // the step's work list, rebuilt when a system joins or leaves it
    int2 *step_map;                        // [k] = (slice, slot) of the k-th listed slice (systems in list order)
    int32_t *step_sys;                     // [k] = slot of the k-th listed system
    int32_t *step_cnt;                     // [0] = listed slices, [1] = listed systems
    int32_t acc32;                         // dot_acc = 1: FP32-phase dot products accumulate in FP32
    int32_t nt;                            // the step product reads the matrices with nontemporal loads
    int32_t hold_above;                    // Algorithm II: a system waits for eps1 at its first crossing when
                                           // more systems than this are listed (else it runs ahead)
};

// One launch's share of a work-list rebuild: entries first .. first + n - 1
// of the list (slot, its first slice and slice count, and the list position
// of its first slice); the last share also writes the totals.
constexpr int kListChunk = 200;   // keeps the launch argument under 4 KB
struct ListChunk {
    int32_t first, n, last, total_slices, total_sys, pad_;
    int32_t slot[kListChunk], slice0[kListChunk], nslices[kListChunk], pre[kListChunk];
};

size_t arena_bytes(int32_t max_sys, int32_t max_slices, int64_t max_entries);
BArena carve(void *base, int32_t max_sys, int32_t max_slices, int64_t max_entries);

// ---- admission, a list of systems per launch ----
// Stage 1 (rows, padded-size scan) needs each system's staged BSys on the
// device; stage 2 (entries, start state, publication) its entry range,
// written into the BSys by the start-state kernel.
constexpr int kAdmitList = 48;   // keeps the argument under 4 KB
struct AdmitList {
    int32_t cnt, pad_;
    int32_t sys[kAdmitList], nsl[kAdmitList], rp_i64[kAdmitList];
    const void *rp[kAdmitList];
    const double *b[kAdmitList];
    const int32_t *col[kAdmitList];
    const double *val[kAdmitList];
    double eps1[kAdmitList];
    int64_t entry0[kAdmitList];
};
void launch_admit_stage1(hipStream_t s, const BArena &a, const AdmitList &l);
void launch_admit_stage2(hipStream_t s, const BArena &a, const AdmitList &l);
void launch_release(hipStream_t s, const BArena &a, int32_t sys, int32_t slice0, int32_t nslices);
void launch_cancel(hipStream_t s, const BArena &a, int32_t sys);       // the solve (step stream)
void launch_bfs_cancel(hipStream_t s, const BArena &a, int32_t sys);   // its 2BFS (BFS stream)
// Algorithm II: eps1 chosen by the host, of candidate class ci (0: 1e-2 ... 5: 1e-7)
void launch_set_eps(hipStream_t s, const BArena &a, int32_t sys, double eps1, int32_t ci);
void launch_fill_slices(hipStream_t s, const BArena &a);   // every slice unowned

// ---- one step over the systems of the work list ----
// A rebuild of the work list (chunks in order); then steps launch grid_slices
// blocks of four slices and grid_sys blocks of one system, at least the
// listed counts (blocks past them return at once).
void launch_worklist(hipStream_t s, const BArena &a, const ListChunk &c);
// dir: some listed system gathers a stored direction (k_b_dir first)
void launch_step(hipStream_t s, const BArena &a, int32_t grid_slices, int32_t grid_sys, bool dir);

// ---- 2BFS (BFS stream) ----
// Kernels on the BFS stream write only the BFS fields of a system's state
// (bfs_*, ncomp, pdiam, small, comp_best, item0) and the BFS arrays; the step
// kernels write the other fields.  Each side's host copy is read only for its
// own fields.
// One round: every system whose sweep is running expands one large level or
// up to small_levels small ones.
// level_grid: blocks of the multi-block level kernel (grid-stride over items);
// small_cap (<= kSmallBfsCap): largest frontier the one-block kernel takes;
// small_work: edge slots (frontier x lanes, summed over levels) after which
// one of its blocks stops, so that wide frontiers do not set the round time.
void launch_bfs_round(hipStream_t s, const BArena &a, int32_t hi_sys, int small_levels, int small_cap,
                      int64_t small_work, int level_grid);
// Band 2BFS of the systems whose entries all lie within |i - j| <= 31 (one
// wave per system, both sweeps in one launch; bit-parallel levels over a
// window of 64 words that follows the frontier).  The system's words of dm
// are formed first (launch_band_masks, one system); the sweeps leave
// bfs_mode = kBfsDone with pdiam, t, u, ncomp = 1, or band_fail set.
constexpr int kBandList = 200;          // systems per launch (keeps the argument under 4 KB)
constexpr int kBandMaxBw = 31;          // offsets d + 32 fit bits 1..63 of a 64-bit mask
// Systems whose entries reach farther than this from the diagonal gather
// scattered columns: their CG product runs in two launches (k_b_dir forms
// d, the product gathers it alone instead of r and d_old).
constexpr int kSplitBw = 4096;
// batch_runahead = 0: systems wait for their features (at their first
// crossing) only while more than this many systems share the steps; with
// fewer, the run-ahead takes bandwidth that would otherwise go unused.
constexpr int kHoldAboveSystems = 8;
struct BandList {
    int32_t cnt, nh_max;                // nh_max: the most offsets of one sign among the listed systems
    int32_t slot[kBandList];
};
void launch_band_masks(hipStream_t s, const BArena &a, int32_t sys, int32_t nslices);
void launch_bfs_band(hipStream_t s, const BArena &a, const BandList &l);
// host-driven transitions of one system of n rows
void launch_bfs_start(hipStream_t s, const BArena &a, int32_t sys, int32_t n);        // CC + sweep-1 seeds
// first sweep from vertex 0 alone, every vertex labelled with it (no
// components): right when the graph is connected, which its end shows
// (reached == n); otherwise the host starts over with launch_bfs_start
void launch_bfs_fast_start(hipStream_t s, const BArena &a, int32_t sys, int32_t n);
void launch_bfs_next_sweep(hipStream_t s, const BArena &a, int32_t sys, int32_t n);   // argmax + sweep-2 seeds
void launch_bfs_finish(hipStream_t s, const BArena &a, int32_t sys, int32_t n);       // argmax + per-system result

// ---- host engine (batch_engine.hip) ----
struct Engine;
Engine *engine_create(int device, const mpcg_options &opt, const mpcg_tuning &tune, const KnnModel *model,
                      void *arena, size_t bytes,
                      int64_t max_rows, int64_t max_entries, int32_t max_sys, int *status);
void engine_destroy(Engine *e);
int engine_submit(Engine *e, const mpcg_request *reqs, int32_t count, uint64_t *ids);
int engine_poll(Engine *e, uint64_t *ids, mpcg_stats *stats, int32_t cap, int32_t *n_done);
int engine_cancel(Engine *e, uint64_t id);
int engine_load(Engine *e, int32_t *queued, int32_t *active);
int64_t engine_max_slices(const Engine *e);
int64_t engine_max_entries(const Engine *e);

}  // namespace batch
}  // namespace mpcg
