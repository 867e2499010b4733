// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "knn.hpp"
#include "mpcg.h"

namespace mpcg {

constexpr int kBlock = 256;           // threads per block of every multi-block kernel
constexpr int kVecPerThread = 4;      // elements per thread in the vector kernels
constexpr int kVecTile = kBlock * kVecPerThread;
constexpr int kK0Max = 64;            // longest FP32 prefix recorded for v
constexpr int kNumEps = 6;            // eps1 candidates 1e-2 ... 1e-7
constexpr int kLdsBytes = 32768;      // LDS staging per SpMV block (val + gathered x)
constexpr int kBfsSmallCap = 2048;    // frontier size handled by the one-workgroup BFS kernel (>= small_max)
constexpr int kBfsSmallThreads = 1024;
constexpr int kBfsSmallWork = 2048;   // (vertex, lane) items per level in the one-workgroup kernel
constexpr int kBfsLevelBlocks = 128;  // level-kernel blocks (measured best on the 128^3 grid)
constexpr int kDiaMax = 16;           // largest number of diagonals the bit-parallel 2BFS handles
constexpr int kDiaRound = 16;         // level launches per round (a multiple of 4: the level rings)
constexpr int kDiaPartMax = 2048;     // largest grid of the level kernels (per-block partials)
constexpr int kDiaTileThreads = 1024; // threads of a temporal-tile block
constexpr int kDiaPerThread = 8;      // words of a tile's loaded range per thread
constexpr int kDiaTileWords = kDiaTileThreads * kDiaPerThread;   // loaded range (LDS: 2 padded copies + visited)
constexpr int kDiaTileDiags = 8;      // most diagonals of a temporal-tile pattern (masks in registers)
constexpr int kDiaPad = 1024;         // zero words beside a tile's LDS range: largest halo per level R
constexpr int kDia2MaxReach = 2048;   // largest R of the two-level kernel (LDS: 2 kBlock + 6 R words)
constexpr int kDiaMaxLevels = 16;     // levels per temporal-tile launch
constexpr int kDiaTileMinLevels = 8;  // fewer levels per launch: the per-level kernel is faster
constexpr int kDiaRing = 64;          // level-count ring (>= 3 launches of levels)
constexpr int64_t kInfinityCacheBytes = 256ll << 20;   // MI355X last-level (Infinity) cache
constexpr int kNumXcd = 8;            // MI355X: blocks are dispatched round-robin over 8 XCDs
constexpr int kMaxGrid = 2048;        // largest grid of a kernel that writes reduction partials
constexpr int kUpdateGrid = 1024;     // blocks of a CG update launch: fewer partials for the next product
constexpr int kSpmvBlocksPerCu = 5;   // 32 KB of LDS per block, 160 KB per CU

enum StopReason : int32_t { kRunning = 0, kConverged = 1, kMaxit = 2, kNotSpd = 3, kNonFinite = 4 };
constexpr int32_t kNoStop = 0x7fffffff;   // DevState::stop_it while the recurrence runs

enum IngestError : int32_t {
    kErrRowPtr = 1, kErrCol = 2, kErrUnsorted = 4, kErrNonFiniteA = 8, kErrNonFiniteB = 16,
    kErrDiag = 32   // Jacobi: a row without a positive, finite diagonal entry
};

// Device-resident solver state: every scalar of the CG recurrence lives here,
// so kernels can be enqueued ahead of the host and stop by themselves.
struct alignas(256) DevState {
    // CG recurrence (FP64 storage; alpha/beta hold the working-precision value)
    double gamma;     // r.r of the current residual (at a stop or a phase start)
    double delta;     // d.(A d) of the last iteration
    double alpha;
    double beta;
    double thr;       // stop when sqrt(gamma) <= thr
    double bnorm2;    // ||b||^2 (FP64)
    double resid2;    // ||b - A x||^2 from the residual kernel
    double gam[2];    // rho_i = r_i.M^-1 r_i by parity of i (= r_i.r_i without a preconditioner);
                      // the product of iteration i writes slot i & 1
    double gr[2];     // r_i.r_i by parity of i (stop test, v ratios)
    double alph[2];   // alpha_i by parity of i (the update of iteration i writes slot i & 1)
    int32_t iter;     // iteration at which the phase started or stopped
    int32_t maxit;
    int32_t live;     // 1 while iterations must continue (read by the host)
    int32_t stop_it;  // the recurrence stopped in iteration stop_it (INT32_MAX while running):
                      // products of later iterations and updates of it and later do nothing
    int32_t x_it;     // x already holds x_{x_it} (set between launches, when a phase starts or
                      // resumes): the product of iteration x_it then has no update to apply
    int32_t reason;   // StopReason
    int32_t k0rec;    // ratios[i] = ||r_{i+1}|| / ||r_i|| is recorded while i < k0rec
    int32_t guard;    // device-side guard tripped (bounded loop exhausted)
    int32_t ing_err;  // IngestError bits
    int32_t max_row;  // longest row seen by the ingest kernel
    int32_t max_band; // largest |i - j| over the stored entries
    int32_t acc32;    // FP32 phase: dot products accumulated in FP32 (dot_acc = 1), else in FP64
    double ratios[kK0Max];
    // BFS.  Launch k of a run expands level bfs_lv[k & 1] (the frontier of
    // level L is queue L & 1, bfs_cnt[L & 3] vertices, smallest bfs_min[L & 3])
    // and hands the next level to launch k + 1 in bfs_lv[(k + 1) & 1]; a level
    // is finished when its launch ends, so no launch needs an arrival count.
    int32_t bfs_lv[2];
    int32_t bfs_cnt[4];
    int32_t bfs_min[4];
    int32_t bfs_done;
    int32_t bfs_ecc;      // largest distance (when done)
    int32_t bfs_far;      // smallest vertex at distance bfs_ecc (when done)
    uint32_t bfs_bar;     // arrivals at the persistent level kernel's grid barrier (cleared per round)
    int64_t bfs_visited;
    int32_t ncomp;
    uint64_t comp_best;   // (ecc << 32) | ~component of the best component
    // Algorithm II run-ahead: while the features are computed, the FP32
    // recurrence continues and x~ is copied the first time sqrt(gamma_i) drops
    // below each candidate threshold spec_thr[t] (t = eps1 class - 2), i >= spec_k0.
    int32_t spec_on, spec_k0;
    int32_t cross_iter[6];
    double spec_thr[6];
    double cross_gamma[6];
    int64_t spare_i64;    // host-side scratch in the pinned mirror
    // Diagonal structure of the pattern (k_dia_offsets): the distinct nonzero
    // offsets j - i of the stored entries, if there are at most kDiaMax
    // (slots filled from 0, 0 = empty; dia_over: more than kDiaMax).
    int32_t dia_base;     // first level of the current round of bit-parallel level launches
    int32_t dia_over;
    int32_t dia_off[16];
};

// Byte offsets of every region inside the caller's arena.
struct Layout {
    size_t state, part, rp32, val32;
    size_t x32, r32, q32, dA32, dB32;
    size_t r64, q64, dA64, dB64;
    size_t dist, q0, q1, label, tarr, best;
    size_t sell_wid, sell_off, sell_col, sell_v64, sell_v32, ingest_blk;
    size_t snap32;      // kNumEps copies of x~ taken at the candidate thresholds
    size_t z32, z64, dg32, dg64;   // Jacobi: M^-1 r and diag(A) in both precisions
    size_t dia_bits;    // bit-parallel 2BFS: frontiers F0, F1, visited V, kDiaMax aligned and kDiaMax row masks
    int64_t sell_cap;   // padded entries the SELL arrays can hold
    size_t total;
    int64_t n, nnz;
};

// Launch shape of the CSR-stream kernels: tiles of R rows, `grid` blocks each
// walking a contiguous range of tiles.
struct SpmvShape {
    int32_t n, R, ntiles, grid;
};
SpmvShape spmv_shape(int64_t n, int64_t nnz, int value_bytes, int num_cu);
int vec_grid(int64_t n);

// SELL-64 copy of A (kernels_sell.hip): slices of 64 rows, entries of a slice
// stored column-major, 16-bit column offsets when the bandwidth allows.
struct SellMat {
    const int32_t *rp;
    const void *scol;
    const double *v64;
    const float *v32;
    const int64_t *off;
    int32_t n, nslices, grid, idx16;
    int32_t batch;   // row entries whose loads are issued together: 4 or 8
    int32_t bf_mask; // whole-batch loads without a guard per entry: bit 0 FP32 kernels, bit 1 FP64
    int32_t nt_mask; // nontemporal loads of the matrix stream: bit 0 FP32 kernels, bit 1 FP64
    int32_t split;   // CG product in two launches (direction, then a one-vector gather)
};

Layout plan_layout(int64_t n, int64_t nnz);

// The matrix as the Jacobi-iteration kernels see it: the SELL-64 copy when the
// solve uses it, else the CSR input (FP32 values from the val32 copy).
struct JacMat {
    const int32_t *rp;
    const int32_t *col;
    int32_t n;
    bool use_sell;
    SellMat sell;
};
int jacobi_grid(const JacMat &m);   // blocks (= partial slots) of one iteration launch
// partials of ||b||^2 into part[np ..], stop markers reset
void launch_jacobi_begin(hipStream_t s, const JacMat &m, const double *b, double *part, DevState *st);
// launch k of a Jacobi stage: x_k in (k & 1 ? x1 : x0) -> x_{k+1}, partials of ||r_k||^2
template <typename T>
void launch_jacobi_iter(hipStream_t s, const JacMat &m, const T *val_csr, const T *b, const T *dg, T *x0, T *x1,
                        int k, int maxit, double eps, int abs_tol, double *part, DevState *st);
void launch_jacobi_widen(hipStream_t s, const float *x32, double *x64, int32_t n);


// Run-ahead test inside the CG product of iteration `it` (FP32 only): returns
// the mask of candidate thresholds first crossed at this iteration (the same in
// every block) and lets block 0 record them; blocks then copy their rows of x~.
__device__ inline unsigned spec_crossings(DevState *st, int it, double g)
{
    if (!st->spec_on || it < st->spec_k0) return 0u;
    unsigned mask = 0u;
    const double rg = sqrt(g);
    for (int t = 0; t < kNumEps; ++t) {
        const int ci = st->cross_iter[t];   // -1, an earlier iteration, or `it` (block 0, this kernel)
        const bool before = ci >= 0 && ci < it;
        if (!before && rg <= st->spec_thr[t]) mask |= 1u << t;
    }
    return mask;
}

// ----- launch wrappers (kernels_cg.hip) -----
// Validate A (and b), convert int64 row pointers, and build the SELL-64 copy
// when its padded size fits in `cap` entries (see kernels_sell.hip).
void launch_ingest_sell(hipStream_t s, const void *rp_in, int rp_is_i64, const int32_t *rp32,
                        int32_t *rp32_out, const int32_t *col, const double *val, const double *b,
                        int32_t n, int64_t nnz, int64_t *wid, int64_t *off, int32_t *blk, int64_t cap,
                        int allow_fill, void *scol, double *sv64, float *sv32, DevState *st);
void launch_cast32(hipStream_t s, const double *val, float *val32, int64_t nnz);
void launch_fill_f64(hipStream_t s, double *p, int64_t n, double v);
void launch_fill_f32(hipStream_t s, float *p, int64_t n, float v);
void launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v);
// FP32 phase start.  Jacobi (dg != nullptr): z = r / dg as well, and the
// phase's rho is r.z; otherwise rho = r.r.
// acc32 = 1: the FP32 phase's dot products (here r~.r~ and r~.z, later d.q,
// r.r, r.z) accumulate in FP32 -- per thread, in the wave and block sums and
// over the block partials -- instead of FP64; recorded in st->acc32 for the
// phase's kernels.
void launch_init32(hipStream_t s, const double *b, float *x, float *r, float *dA, int32_t n,
                   double eps, int abs_tol, int32_t maxit, int32_t k0rec, const float *dg, float *z,
                   double *part, DevState *st, int acc32);
// Jacobi: dg64 = diag(A), dg32 = float32(dg64); a row without a positive,
// finite diagonal entry sets kErrDiag.
void launch_diag(hipStream_t s, const int32_t *rp, const int32_t *col, const double *val, int32_t n,
                 double *dg64, float *dg32, DevState *st);
void launch_set_phase(hipStream_t s, DevState *st, double thr, int32_t maxit, int32_t k0rec);
// Start the run-ahead: thresholds eps_t * scale, first test at iteration k0.
void launch_set_spec(hipStream_t s, DevState *st, double scale, int32_t k0, int32_t maxit);
void launch_timing_state(hipStream_t s, DevState *st, double *part, int cnt);
// CG iteration `it` of a phase that started at `it0`: product kernel (reads the
// update partials `up`, writes its own to `part`) and update kernel (reads
// `sp`, writes `up`).
// The product of iteration it > it0 also applies the previous iteration's
// x += alpha_{it-1} d_{it-1} (deferred from the update, which then needs
// neither x nor d), and copies the updated x~ into `snap` at a run-ahead
// crossing (FP32 only).
// `r` is the vector the direction is built from: the residual, or z = M^-1 r
// with Jacobi (pc = 1, the update partials then hold rho and r.r).
template <typename T>
void launch_cg_spmv(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                    const T *val, const T *r, T *dA, T *dB, T *q, const double *up, int nup,
                    double *part, int it, int it0, T *x, T *snap, int pc, DevState *st);
// Jacobi (dg != nullptr): also z = r / dg and partials of r.z (slot 0) and r.r
// (slot nup + block).
template <typename T>
void launch_cg_update(hipStream_t s, int32_t n, T *r, const T *q, const double *sp, int nsp, double *up,
                      int nup, int it, const T *dg, T *z, DevState *st);
// r = b - A x (x from float x32 when x32 != nullptr, else from x64), x64 <- float64(x32),
// zero the old-direction buffer of iteration it0, gamma = r.r, ||b||^2, stop test.
// Jacobi (dg != nullptr): z = r / dg; the partials are r.r, b.b and r.z (r.r
// again without a preconditioner), three per block.
void launch_restart(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                    const double *val, const float *x32, double *x64, const double *b, double *r,
                    double *dA, double *dB, int it0, double eps, int abs_tol, int32_t maxit,
                    const double *dg, double *z, double *part, DevState *st);
void launch_resid(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                  const double *val, const double *x64, const double *b, double *part, DevState *st);
void launch_fin_restart(hipStream_t s, const double *part, int cnt, int it0, double eps, int abs_tol,
                        int32_t maxit, DevState *st);
void launch_fin_resid(hipStream_t s, const double *part, int cnt, DevState *st);
template <typename T>
void launch_spmv_plain(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                       const T *val, const T *x, T *y);

// ----- SELL-64 (kernels_sell.hip) -----
template <typename T>
void launch_sell_cg_spmv(hipStream_t s, const SellMat &m, const T *r, T *dA, T *dB, T *q,
                         const double *up, int nup, double *part, int it, int it0, T *x, T *snap, int pc,
                         DevState *st);
void launch_sell_restart(hipStream_t s, const SellMat &m, const float *x32, double *x64,
                         const double *b, double *r, double *dA, double *dB, int it0, const double *dg,
                         double *z, double *part, DevState *st);
void launch_sell_resid(hipStream_t s, const SellMat &m, const double *x64, const double *b,
                       double *part, DevState *st);
template <typename T>
void launch_sell_plain(hipStream_t s, const SellMat &m, const T *x, T *y);

// ----- BFS (kernels_bfs.hip) -----
// A queued BFS vertex is stored as its CSR row range: the level that expands
// it needs no further load to find its neighbours.
struct QEnt {
    int32_t b, e;
};

// The diagonals of a pattern (offsets j - i, nd of them), passed by value.
struct DiaOffs {
    int32_t d[kDiaMax];
    int32_t q[kDiaMax], r[kDiaMax];   // -d = 32 q + r, 0 <= r < 32 (window word and shift)
    int32_t nd;
};

struct BfsBufs {
    const int32_t *rp, *col;
    int32_t n;
    int32_t lanes;          // lanes per frontier vertex in the one-workgroup kernel
    int32_t small_max;      // largest frontier left to the one-workgroup kernel
    int32_t band;           // largest |i - j| over the stored entries (window placement)
    int32_t *dist, *label, *tarr;
    QEnt *q0, *q1;      // frontier queues: the row range of each queued vertex
    unsigned long long *best;
    DevState *st;
    int32_t grid;       // blocks of the level kernel
    int32_t precheck;   // read the distance before claiming a vertex
    int32_t persist;    // large levels in one persistent launch (grid barrier) instead of one launch each
    // bit-parallel levels over the diagonals (when the pattern has at most
    // kDiaMax of them): frontier bits of even / odd levels, visited bits, and
    // per diagonal t the rows v that row v - d_t reaches (aligned masks)
    int32_t dia;        // 1: the sweeps run as bit-parallel levels
    int32_t nwords;     // 32-bit words per bit vector
    int32_t dia_grid;   // largest grid of the level kernel
    DiaOffs doff;       // the diagonals (host copy of st->dia_off)
    uint32_t *df0, *df1, *dv, *dm, *draw;   // dm, draw: kDiaMax masks of nwords words each
    // temporal tiles: dia_h levels per launch, dia_T words per block, halo
    // dia_R words per level (dia_h = 0: one level per launch)
    int32_t dia_h, dia_T, dia_R;
    int32_t *ring_cnt, *ring_min;   // kDiaRing slots each
    int32_t *part_cnt, *part_min;   // level kernels: 2 parities x 2 levels x kDiaPartMax per-block partials each
    int32_t dia_two;                // two levels per launch (k_dia_level2)
};
// Diagonal structure: st->dia_over / dia_off from the CSR pattern (cleared
// first); then, with b.doff filled from them, the masks.  Columns outside
// [0, n) are ignored.
void launch_dia_detect(hipStream_t s, const BfsBufs &b);
void launch_dia_masks(hipStream_t s, const BfsBufs &b);
// Single-source sweep with bit-parallel levels: seed, then rounds of
// kDiaRound level launches and one that moves the round's base level on;
// every launch of a round has fixed arguments (the queue kernels'
// level-state protocol).
void launch_dia_seed(hipStream_t s, const BfsBufs &b, int32_t src);
void launch_dia_round(hipStream_t s, const BfsBufs &b);
// Temporal tiles: the ring's seed (after launch_dia_seed), then rounds of
// `launches` launches of dia_h levels each; launch k expands levels
// k dia_h .. (k + 1) dia_h - 1.
void launch_dia_ring_seed(hipStream_t s, const BfsBufs &b, int32_t src);
int launch_dia_multi_round(hipStream_t s, const BfsBufs &b, int launches, int k);
void launch_bfs_seed_single(hipStream_t s, const BfsBufs &b, int32_t src);
// Enqueues one round (the one-workgroup kernel, then `levels` level kernels)
// with launch indices k, k + 1, ...; returns the next launch index.
int launch_bfs_round(hipStream_t s, const BfsBufs &b, int levels, int k);

void launch_cc(hipStream_t s, const BfsBufs &b);
// hist[d] += number of vertices at distance d >= 1 (hist must hold the largest distance + 1)
void launch_dist_hist(hipStream_t s, const int32_t *dist, int32_t n, unsigned long long *hist);
void launch_bfs_seed_roots(hipStream_t s, const BfsBufs &b);
void launch_comp_argmax(hipStream_t s, const BfsBufs &b, int second_sweep);
void launch_bfs_seed_far(hipStream_t s, const BfsBufs &b);
void launch_comp_final(hipStream_t s, const BfsBufs &b);

}  // namespace mpcg
