// Kernels of the batched engine (gfx950, wave64).  The layout and the step
// are described in batch_internal.hpp.  Per system the arithmetic is the one
// of the single-system path: the CG procedure of the paper's "Conjugate
// Gradient Method" section in FP32 (dots accumulated in FP64, alpha and beta
// rounded to FP32), the restart of Algorithm I step 5 (float64(x~), residual
// b - A x in FP64), the FP64 phase, the final true-residual check, and the
// 2BFS of the section "Computing Pseudo-Diameter of the Graph Matrix" per
// connected component.

#include "batch_internal.hpp"

#include <cmath>

namespace mpcg {
namespace batch {

namespace {

constexpr int kIntMax = 0x7fffffff;
constexpr int kLoadBatch = 4;

template <typename T> __device__ inline T fma_b(T a, T b, T c);
template <> __device__ inline float fma_b<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ inline double fma_b<double>(double a, double b, double c) { return fma(a, b, c); }

__device__ inline double wave_sum_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int wave_max_i32(int v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}

// Fixed-order block sum (kBlock threads); the result is valid in thread 0.
__device__ inline double block_sum_d(double v, double *sm)
{
    v = wave_sum_d(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += sm[i];
    __syncthreads();
    return s;
}

// Sum of component j of the slice partials of system S, fixed order.
__device__ inline double sys_sum(const BArena &a, const BSys &S, int j, double *sm)
{
    // four loads in flight per thread, added in index order (the same bits
    // as one at a time)
    const double *p = a.pslice + 2 * (size_t)S.slice0 + j;
    const int cnt = S.nslices;
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < cnt; i += 4 * kBlock) {
        const double p0 = p[2 * (size_t)i], p1 = p[2 * (size_t)(i + kBlock)];
        const double p2 = p[2 * (size_t)(i + 2 * kBlock)], p3 = p[2 * (size_t)(i + 3 * kBlock)];
        acc += p0;
        acc += p1;
        acc += p2;
        acc += p3;
    }
    for (; i < cnt; i += kBlock) acc += p[2 * (size_t)i];
    return block_sum_d(acc, sm);
}

// dot_acc = 1: the FP32 phase's sums in float (partials stored widened, exact).
__device__ inline float wave_sum_f(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double sys_sum_f(const BArena &a, const BSys &S, int j, double *sm)
{
    const double *p = a.pslice + 2 * (size_t)S.slice0 + j;
    const int cnt = S.nslices;
    float acc = 0.0f;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < cnt; i += 4 * kBlock) {
        const double p0 = p[2 * (size_t)i], p1 = p[2 * (size_t)(i + kBlock)];
        const double p2 = p[2 * (size_t)(i + 2 * kBlock)], p3 = p[2 * (size_t)(i + 3 * kBlock)];
        acc += (float)p0;
        acc += (float)p1;
        acc += (float)p2;
        acc += (float)p3;
    }
    for (; i < cnt; i += kBlock) acc += (float)p[2 * (size_t)i];
    acc = wave_sum_f(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = (double)acc;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += (float)sm[i];
    __syncthreads();
    return (double)s;
}

// A partial of an FP32-phase dot product in the precision dot_acc asks for:
// the lane's term (exact in FP64, one rounding in FP32) summed over the wave.
__device__ inline double wave_dot32(bool f32, float x, float y)
{
    return f32 ? (double)wave_sum_f(x * y) : wave_sum_d((double)x * (double)y);
}

__device__ inline int64_t rp_at(const void *rp, int i64, int64_t i)
{
    return i64 ? static_cast<const int64_t *>(rp)[i] : (int64_t) static_cast<const int32_t *>(rp)[i];
}

}  // namespace

// ---------------------------------------------------------------- arena --

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t arena_bytes(int32_t max_sys, int32_t max_slices, int64_t max_entries)
{
    const size_t rows = (size_t)max_slices * 64, sl = (size_t)max_slices, e = (size_t)max_entries;
    size_t t = 0;
    t += up256(sizeof(BSys) * (size_t)max_sys);
    t += up256(4 * sl) * 2 + up256(8 * sl) + up256(16 * sl);          // slice_w, sys_of_slice, slice_off, pslice
    t += up256(4 * rows);                                             // rowlen
    t += up256(8 * rows) * 6 + up256(4 * rows) * 5;                   // FP64 and FP32 vectors
    t += up256(4 * rows * kNumEps);                                   // run-ahead copies of x~
    t += up256(4 * rows) * 5 + up256(8 * rows) + up256(rows / 8);     // BFS
    t += up256(8 * rows);                                             // band 2BFS masks
    t += up256(4 * e) + up256(8 * e) + up256(4 * e);                  // col, v64, v32
    t += up256(4 * (size_t)max_sys) * 2 + up256(8 * (size_t)max_sys) + 256 + 256;
    t += up256(8 * sl) + up256(4 * (size_t)max_sys) + 256;            // step work list
    return t;
}

BArena carve(void *base, int32_t max_sys, int32_t max_slices, int64_t max_entries)
{
    BArena a{};
    char *p = static_cast<char *>(base);
    const size_t rows = (size_t)max_slices * 64, sl = (size_t)max_slices, e = (size_t)max_entries;
    auto take = [&](size_t bytes) { char *q = p; p += up256(bytes); return q; };
    a.max_sys = max_sys;
    a.max_slices = max_slices;
    a.max_entries = max_entries;
    a.sys = reinterpret_cast<BSys *>(take(sizeof(BSys) * (size_t)max_sys));
    a.slice_w = reinterpret_cast<int32_t *>(take(4 * sl));
    a.sys_of_slice = reinterpret_cast<int32_t *>(take(4 * sl));
    a.slice_off = reinterpret_cast<int64_t *>(take(8 * sl));
    a.pslice = reinterpret_cast<double *>(take(16 * sl));
    a.rowlen = reinterpret_cast<int32_t *>(take(4 * rows));
    a.b64 = reinterpret_cast<double *>(take(8 * rows));
    a.x64 = reinterpret_cast<double *>(take(8 * rows));
    a.r64 = reinterpret_cast<double *>(take(8 * rows));
    a.q64 = reinterpret_cast<double *>(take(8 * rows));
    a.dA64 = reinterpret_cast<double *>(take(8 * rows));
    a.dB64 = reinterpret_cast<double *>(take(8 * rows));
    a.x32 = reinterpret_cast<float *>(take(4 * rows));
    a.r32 = reinterpret_cast<float *>(take(4 * rows));
    a.q32 = reinterpret_cast<float *>(take(4 * rows));
    a.dA32 = reinterpret_cast<float *>(take(4 * rows));
    a.dB32 = reinterpret_cast<float *>(take(4 * rows));
    a.snap32 = reinterpret_cast<float *>(take(4 * rows * kNumEps));
    a.dist = reinterpret_cast<int32_t *>(take(4 * rows));
    a.q0 = reinterpret_cast<int32_t *>(take(4 * rows));
    a.q1 = reinterpret_cast<int32_t *>(take(4 * rows));
    a.label = reinterpret_cast<int32_t *>(take(4 * rows));
    a.tarr = reinterpret_cast<int32_t *>(take(4 * rows));
    a.best = reinterpret_cast<unsigned long long *>(take(8 * rows));
    a.vis = reinterpret_cast<uint32_t *>(take(rows / 8));
    a.dm = reinterpret_cast<uint32_t *>(take(8 * rows));
    a.col = reinterpret_cast<int32_t *>(take(4 * e));
    a.v64 = reinterpret_cast<double *>(take(8 * e));
    a.v32 = reinterpret_cast<float *>(take(4 * e));
    a.act_sys = reinterpret_cast<int32_t *>(take(4 * (size_t)max_sys));
    a.small_sys = reinterpret_cast<int32_t *>(take(4 * (size_t)max_sys));
    a.act_pre = reinterpret_cast<int64_t *>(take(8 * (size_t)max_sys));
    a.counts = reinterpret_cast<int32_t *>(take(256));
    a.items = reinterpret_cast<int64_t *>(take(256));
    a.step_map = reinterpret_cast<int2 *>(take(8 * sl));
    a.step_sys = reinterpret_cast<int32_t *>(take(4 * (size_t)max_sys));
    a.step_cnt = reinterpret_cast<int32_t *>(take(256));
    return a;
}

// ------------------------------------------------------------ admission --

__device__ inline void adm_fill(const BArena &a, int32_t slice0, int32_t nslices, int blk)
{
    const int j = blk * kBlock + threadIdx.x;
    if (j < nslices) a.slice_w[slice0 + j] = 0;
}

__global__ void k_fill_slices(BArena a)
{
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.max_slices; j += gridDim.x * kBlock)
        a.sys_of_slice[j] = -1;
}

void launch_fill_slices(hipStream_t s, const BArena &a)
{
    int g = (a.max_slices + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_slices, dim3(g < 1 ? 1 : g), dim3(kBlock), 0, s, a);
}

// Thread per (padded) row of the system: row length, slice width, b, the FP32
// start r~ = float32(b), x = 0, and per-slice partials of r~.r~ and b.b.
__device__ inline void adm_rows(const BArena &a, int32_t sys, const void *rp, int rp_i64, const double *b,
                                int32_t row0, int32_t n, int64_t nnz, int32_t slice0, int32_t nslices, int blk)
{
    const int64_t i = (int64_t)blk * kBlock + threadIdx.x;   // local row
    if (i >= (int64_t)nslices * 64) return;
    const int64_t g = row0 + i;
    int err = 0, len = 0;
    double bv = 0.0;
    if (i < n) {
        const int64_t lo = rp_at(rp, rp_i64, i), hi = rp_at(rp, rp_i64, i + 1);
        if (i == 0 && lo != 0) err |= kErrRowPtr;
        if (i == n - 1 && hi != nnz) err |= kErrRowPtr;
        if (lo < 0 || hi < lo || hi > nnz || hi - lo > 0x7fffffff) err |= kErrRowPtr;
        else len = (int)(hi - lo);
        bv = b[i];
        if (!isfinite(bv)) err |= kErrNonFiniteB;
    }
    a.rowlen[g] = len;
    a.b64[g] = bv;
    a.x64[g] = 0.0;
    a.x32[g] = 0.0f;
    const float rv = (float)bv;
    a.r32[g] = rv;
    a.r64[g] = 0.0;
    a.q64[g] = 0.0;
    a.q32[g] = 0.0f;
    a.dA64[g] = 0.0;
    a.dB64[g] = 0.0;
    a.dA32[g] = 0.0f;
    a.dB32[g] = 0.0f;
    const int sl = slice0 + (int)(i >> 6);
    if (len > 0) atomicMax(&a.slice_w[sl], len);
    const double pr = wave_dot32(a.acc32, rv, rv);
    const double pb = wave_sum_d(bv * bv);
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if ((threadIdx.x & 63) == 0) {
        a.pslice[2 * (size_t)sl] = pr;
        a.pslice[2 * (size_t)sl + 1] = pb;
        a.sys_of_slice[sl] = -1;   // not visible to the step kernels until the system is complete
        if (err) atomicOr(&a.sys[sys].err, err);
    }
}

// Padded entry offsets of the system's slices (local to its entry range).
__device__ inline void adm_scan(const BArena &a, int32_t sys, int64_t *part)
{
    BSys &S = a.sys[sys];
    const int ns = S.nslices, s0 = S.slice0;
    const int per = (ns + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, ns);
    int64_t acc = 0;
    for (int j = b0; j < b1; ++j) acc += (int64_t)a.slice_w[s0 + j] * 64;
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        S.padded = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int j = b0; j < b1; ++j) {
        a.slice_off[s0 + j] = run;
        run += (int64_t)a.slice_w[s0 + j] * 64;
    }
}

// Wave per slice: column range, strictly increasing columns and finite
// values checked; entries written column-major inside the slice with global
// column indices.  Lanes past a row's length get a zero entry on their own
// row, which the products never read (they stop at the row length).
__device__ inline void adm_entries(const BArena &a, int32_t sys, const void *rp, int rp_i64, const int32_t *col,
                                   const double *val, int64_t entry0, int blk)
{
    const BSys &S = a.sys[sys];
    const int lane = threadIdx.x & 63;
    const int j = blk * kSlicesPerBlock + (threadIdx.x >> 6);
    if (j >= S.nslices) return;
    const int sl = S.slice0 + j;
    const int64_t i = (int64_t)j * 64 + lane;
    const int64_t g = S.row0 + i;
    const int W = a.slice_w[sl];
    const int64_t base = entry0 + a.slice_off[sl] + lane;
    const int len = a.rowlen[g];
    const int64_t lo = i < S.n ? rp_at(rp, rp_i64, i) : 0;
    int err = 0, prev = -1, bw = 0;
    unsigned long long offs = 0ull;   // the band 2BFS's offsets
    for (int k = 0; k < W; ++k) {
        int cg = (int)g;
        double v = 0.0;
        if (k < len && lo >= 0 && lo + k < S.nnz) {   // rows with bad pointers have len 0 already
            const int c = col[lo + k];
            v = val[lo + k];
            if (c < 0 || c >= S.n) err |= kErrCol;
            else if (c <= prev) err |= kErrUnsorted;
            if (!isfinite(v)) err |= kErrNonFiniteA;
            prev = c;
            cg = S.row0 + (c >= 0 && c < S.n ? c : 0);
            const int d = cg - (int)g;
            const int ad = d < 0 ? -d : d;
            bw = ad > bw ? ad : bw;
            if (d != 0 && ad <= kBandMaxBw) offs |= 1ull << (d + 32);
        }
        a.col[base + (int64_t)k * 64] = cg;
        a.v64[base + (int64_t)k * 64] = v;
        a.v32[base + (int64_t)k * 64] = (float)v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        err |= __shfl_xor(err, o, 64);
        const int b2 = __shfl_xor(bw, o, 64);
        bw = b2 > bw ? b2 : bw;
        offs |= __shfl_xor(offs, o, 64);
    }
    if (lane == 0) {
        if (err) atomicOr(&a.sys[sys].err, err);
        if (bw) atomicMax(&a.sys[sys].bw, bw);
        if (offs) atomicOr(&a.sys[sys].doffs, offs);
    }
}

// Start state.  Host-filled fields (options, ranges) are already in place.
__device__ inline void adm_finish(const BArena &a, int32_t sys, double eps1, int64_t entry0, double *sm)
{
    BSys &S = a.sys[sys];
    const double g0 = a.acc32 ? sys_sum_f(a, S, 0, sm) : sys_sum(a, S, 0, sm);
    const double bb = sys_sum(a, S, 1, sm);
    if (threadIdx.x == 0) {
        S.entry0 = entry0;
        S.split = S.bw > kSplitBw ? 1 : 0;   // the entries' pass has recorded the bandwidth
        S.bb = bb;
        S.gamma = g0;
        S.ph_it = 0;
        S.n1 = S.n2 = 0;
        S.restarts = 0;
        S.upd = 0;
        const double sb = sqrt(bb);
        S.thr2 = S.tol_abs ? S.eps2 : S.eps2 * sb;
        double e = 1e-2;
        for (int t = 0; t < kNumEps; ++t, e *= 0.1) {
            S.spec_thr[t] = S.tol_abs ? e : e * sb;
            S.cross_iter[t] = -1;
            S.cross_gamma[t] = 0.0;
        }
        S.snap_mask = 0;
        S.ra_stop = kRaNone;
        if (S.err) {
            S.status = (S.err & (kErrNonFiniteA | kErrNonFiniteB)) ? MPCG_ENONFINITE : MPCG_EINVAL;
            S.mode = kDone;
        } else if (bb == 0.0) {
            S.status = MPCG_OK;
            S.mode = kDone;
        } else if (eps1 == MPCG_EPS1_NONE) {
            S.src = kSrcZero;
            S.mode = kRestart;
        } else {
            S.eps_set = S.auto_eps ? 0 : 1;
            S.thr1 = S.auto_eps ? 0.0 : (S.tol_abs ? eps1 : eps1 * sb);
            if (S.auto_eps) {
                S.mode = g0 == 0.0 ? kHold : kCg32;
            } else if (sqrt(g0) <= S.thr1) {
                S.relres_sp = sqrt(g0) / sb;
                S.src = kSrcX32;
                S.mode = kRestart;
            } else {
                S.mode = kCg32;
            }
        }
    }
}

// Marks the system's slices as live (after every admission kernel).
__device__ inline void adm_publish(const BArena &a, int32_t sys, int blk)
{
    const BSys &S = a.sys[sys];
    const int j = blk * kBlock + threadIdx.x;
    if (j < S.nslices) a.sys_of_slice[S.slice0 + j] = sys;
}

// ---- admission of a list of systems: one launch per stage ----
//
// The blocks of a launch are dealt to the listed systems in order, each
// system taking as many as its slices need (spb slices per block); a block
// finds its system by walking the list (at most kAdmitList entries).
__device__ inline bool adm_block(const AdmitList &L, int spb, int &j, int &blk)
{
    int b = (int)blockIdx.x;
    for (j = 0; j < L.cnt; ++j) {
        const int nb = (L.nsl[j] + spb - 1) / spb;
        if (b < nb) {
            blk = b;
            return true;
        }
        b -= nb;
    }
    return false;
}

// stage 1: slice widths zeroed (a launch of its own: the rows' pass takes
// their maximum), then the rows' pass, then the padded-size scan
__global__ void __launch_bounds__(kBlock) k_admit_fill_l(BArena a, AdmitList L)
{
    int j, blk;
    if (!adm_block(L, kBlock, j, blk)) return;
    const BSys &S = a.sys[L.sys[j]];
    adm_fill(a, S.slice0, S.nslices, blk);
}

__global__ void __launch_bounds__(kBlock) k_admit_rows_l(BArena a, AdmitList L)
{
    int j, blk;
    if (!adm_block(L, kSlicesPerBlock, j, blk)) return;
    const BSys &S = a.sys[L.sys[j]];
    adm_rows(a, L.sys[j], L.rp[j], L.rp_i64[j], L.b[j], S.row0, S.n, S.nnz, S.slice0, S.nslices, blk);
}

__global__ void __launch_bounds__(1024) k_admit_scan_l(BArena a, AdmitList L)
{
    __shared__ int64_t part[1024];
    if ((int)blockIdx.x >= L.cnt) return;
    adm_scan(a, L.sys[blockIdx.x], part);
}

// stage 2: entries, start state (block per system), publication
__global__ void __launch_bounds__(kBlock) k_admit_entries_l(BArena a, AdmitList L)
{
    int j, blk;
    if (!adm_block(L, kSlicesPerBlock, j, blk)) return;
    adm_entries(a, L.sys[j], L.rp[j], L.rp_i64[j], L.col[j], L.val[j], L.entry0[j], blk);
}

__global__ void __launch_bounds__(kBlock) k_admit_finish_l(BArena a, AdmitList L)
{
    __shared__ double sm[kBlock / 64 + 1];
    if ((int)blockIdx.x >= L.cnt) return;
    adm_finish(a, L.sys[blockIdx.x], L.eps1[blockIdx.x], L.entry0[blockIdx.x], sm);
}

__global__ void __launch_bounds__(kBlock) k_admit_publish_l(BArena a, AdmitList L)
{
    int j, blk;
    if (!adm_block(L, kBlock, j, blk)) return;
    adm_publish(a, L.sys[j], blk);
}

__global__ void k_release(BArena a, int32_t sys, int32_t slice0, int32_t nslices)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nslices; j += gridDim.x * blockDim.x)
        a.sys_of_slice[slice0 + j] = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.sys[sys].mode = kFree;
        a.sys[sys].bfs_mode = kBfsNone;
    }
}

__global__ void k_cancel(BArena a, int32_t sys)
{
    if (threadIdx.x == 0) {
        BSys &S = a.sys[sys];
        S.mode = kDone;
        S.status = MPCG_ECANCELED;
        S.upd = 0;
    }
}

// Stops the system's 2BFS: the next rounds skip it.
__global__ void k_bfs_cancel(BArena a, int32_t sys)
{
    if (threadIdx.x == 0) {
        BSys &S = a.sys[sys];
        if (S.bfs_mode == kBfsRun || S.bfs_mode == kBfsSwept) S.bfs_mode = kBfsNone;
    }
}

// Algorithm II: eps1 (candidate class ci) from the kNN choice.  A system
// still in its k0 prefix picks the eps1 test up when the prefix ends.  One
// past it has been running ahead: if it crossed eps1 on the way, the FP64
// restart starts from the copy of x~ at that first crossing (or from x~
// itself while that copy is still due: x~ has not moved since); if the run
// stopped (breakdown, maxit1) before reaching eps1, from x~ at the stop;
// otherwise the FP32 phase continues with the eps1 test (Remark 3).  Each
// case is the state the sequential method stops in.
__global__ void k_set_eps(BArena a, int32_t sys, double eps1, int32_t ci)
{
    if (threadIdx.x != 0) return;
    BSys &S = a.sys[sys];
    const double sb = sqrt(S.bb);
    S.thr1 = S.tol_abs ? eps1 : eps1 * sb;
    S.eps_set = 1;
    if (S.mode == kHold && S.k0_used == 0) {   // gamma_0 = 0 at admission: nothing to iterate
        S.relres_sp = sqrt(S.gamma) / sb;
        S.src = kSrcX32;
        S.ph_it = 0;
        S.mode = kRestart;
        return;
    }
    if (S.spec) {   // the speculative FP64 phase (see k_b_scalar2)
        S.spec = 0;
        if (ci >= 0 && ci < kNumEps && S.cross_iter[ci] == S.cross_iter[kNumEps - 1]) return;   // same state: kept
        // discarded: the FP64 stage starts again from the chosen candidate's copy
        S.n2 = 0;
        S.restarts = 0;
        S.flags &= ~MPCG_FLAG_FINAL_RESTARTED;
        S.pend = 0;
        S.status = MPCG_OK;
        S.n1 = S.cross_iter[ci];
        S.gamma = S.cross_gamma[ci];
        S.relres_sp = sqrt(S.gamma) / sb;
        S.src = ((S.snap_mask >> ci) & 1) ? kSrcX32 : kSrcSnap;
        S.snap_ci = ci;
        S.upd = 0;
        S.ph_it = 0;
        S.mode = kRestart;
        return;
    }
    if (S.k0_used == 0 || (S.mode != kHold && S.mode != kCg32)) return;
    if (ci >= 0 && ci < kNumEps && S.cross_iter[ci] >= 0) {
        S.n1 = S.cross_iter[ci];
        S.gamma = S.cross_gamma[ci];
        S.relres_sp = sqrt(S.gamma) / sb;
        S.src = ((S.snap_mask >> ci) & 1) ? kSrcX32 : kSrcSnap;
        S.snap_ci = ci;
        S.upd = 0;
        S.ph_it = 0;
        S.mode = kRestart;
    } else if (S.mode == kHold && S.ra_stop == kRaWait) {
        // held right after the k0 prefix, eps1 not yet crossed: the FP32
        // phase continues with the eps1 test
        S.ra_stop = kRaNone;
        S.mode = kCg32;
    } else if (S.mode == kHold) {
        S.flags |= S.ra_stop == kRaBreakdown ? MPCG_FLAG_FP32_BREAKDOWN : MPCG_FLAG_FP32_MAXIT;
        S.relres_sp = sqrt(S.gamma) / sb;
        S.src = kSrcX32;
        S.ph_it = 0;
        S.mode = kRestart;
    }
}

// ----------------------------------------------------------------- step --

// NT: nontemporal loads of the matrix stream (an arena beyond the Infinity
// Cache: streamed once per step, the matrices then do not evict the vectors)
template <bool NT, typename P> __device__ inline P b_ld(const P *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// Wave per slice.  CG product of iteration j of the phase:
// d_j = r_j + beta_j d_{j-1} (d_0 = r_0), q = A d_j, partial of d_j.q (FP64).
template <typename T, bool NT>
__device__ inline double cg_product(const BArena &a, const BSys &S, const T *val, const T *r, T *dA, T *dB,
                                    T *q, int64_t base, int row, int len)
{
    const int j = S.ph_it;
    const bool first = j == 0;
    const T beta = (T)S.beta;
    T *dnew = (j & 1) ? dB : dA;
    const T *dold = (j & 1) ? dA : dB;
    if (S.split) {   // d_j was formed by k_b_dir: gather it alone
        T acc = T(0);
        const int W = wave_max_i32(len);
        for (int k0 = 0; k0 < W; k0 += kLoadBatch) {
            int c[kLoadBatch];
            T v[kLoadBatch], g[kLoadBatch];
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t)
                if (k0 + t < len) {
                    c[t] = b_ld<NT>(a.col + base + (int64_t)(k0 + t) * 64);
                    v[t] = b_ld<NT>(val + base + (int64_t)(k0 + t) * 64);
                }
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t)
                if (k0 + t < len) g[t] = dnew[c[t]];
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t)
                if (k0 + t < len) acc = fma_b<T>(v[t], g[t], acc);
        }
        const T dn = dnew[row];
        q[row] = acc;
        if (sizeof(T) == 4 && a.acc32) return (double)wave_sum_f((float)dn * (float)acc);
        return wave_sum_d((double)dn * (double)acc);
    }
    T acc = T(0);
    const int W = wave_max_i32(len);
    for (int k0 = 0; k0 < W; k0 += kLoadBatch) {
        int c[kLoadBatch];
        T v[kLoadBatch], g[kLoadBatch];
        if (sizeof(T) == 4) {
            // FP32: every lane loads the whole batch (the padding entries are
            // zero entries on the lane's own row; past W the last column is
            // read again), so the batch's loads and its gathers are issued
            // together; only the products past the row's length are skipped
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t) {
                const int kk = k0 + t < W ? k0 + t : W - 1;
                c[t] = b_ld<NT>(a.col + base + (int64_t)kk * 64);
                v[t] = b_ld<NT>(val + base + (int64_t)kk * 64);
            }
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t) g[t] = first ? r[c[t]] : fma_b<T>(beta, dold[c[t]], r[c[t]]);
        } else {
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t)
                if (k0 + t < len) {
                    c[t] = b_ld<NT>(a.col + base + (int64_t)(k0 + t) * 64);
                    v[t] = b_ld<NT>(val + base + (int64_t)(k0 + t) * 64);
                }
#pragma unroll
            for (int t = 0; t < kLoadBatch; ++t)
                if (k0 + t < len) g[t] = first ? r[c[t]] : fma_b<T>(beta, dold[c[t]], r[c[t]]);
        }
#pragma unroll
        for (int t = 0; t < kLoadBatch; ++t)
            if (k0 + t < len) acc = fma_b<T>(v[t], g[t], acc);
    }
    const T dn = first ? r[row] : fma_b<T>(beta, dold[row], r[row]);
    dnew[row] = dn;
    q[row] = acc;
    if (sizeof(T) == 4 && a.acc32) return (double)wave_sum_f((float)dn * (float)acc);   // already summed
    return wave_sum_d((double)dn * (double)acc);
}

// Restart: r = b - A x with x = float64(x~), x, or 0; x takes that value.
// Final check: partial of ||b - A x||^2.
template <bool NT>
__device__ inline double residual(const BArena &a, const BSys &S, bool restart, int64_t base, int row, int len)
{
    const int src = restart ? S.src : kSrcX64;
    const float *xs = a.snap32 + (size_t)S.snap_ci * ((size_t)a.max_slices * 64);   // src == kSrcSnap
    double acc = 0.0;
    const int W = wave_max_i32(len);
    for (int k0 = 0; k0 < W; k0 += kLoadBatch) {
        int c[kLoadBatch];
        double v[kLoadBatch], g[kLoadBatch];
#pragma unroll
        for (int t = 0; t < kLoadBatch; ++t)
            if (k0 + t < len) {
                c[t] = b_ld<NT>(a.col + base + (int64_t)(k0 + t) * 64);
                v[t] = b_ld<NT>(a.v64 + base + (int64_t)(k0 + t) * 64);
            }
#pragma unroll
        for (int t = 0; t < kLoadBatch; ++t)
            if (k0 + t < len)
                g[t] = src == kSrcX32   ? (double)a.x32[c[t]]
                       : src == kSrcSnap ? (double)xs[c[t]]
                       : src == kSrcX64  ? a.x64[c[t]]
                                         : 0.0;
#pragma unroll
        for (int t = 0; t < kLoadBatch; ++t)
            if (k0 + t < len) acc = fma(v[t], g[t], acc);
    }
    const double res = a.b64[row] - acc;
    if (restart) {
        if (src == kSrcX32) a.x64[row] = (double)a.x32[row];
        else if (src == kSrcSnap) a.x64[row] = (double)xs[row];
        else if (src == kSrcZero) a.x64[row] = 0.0;
        a.r64[row] = res;
    }
    return res * res;
}

template <bool NT>
__global__ void __launch_bounds__(kBlock) k_b_product(BArena a)
{
    const int k = blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
    if (k >= a.step_cnt[0]) return;
    const int2 e = a.step_map[k];   // slice and its system: no dependent lookup of the owner
    const int sl = e.x, s = e.y;
    if (s < 0) return;
    const BSys &S = a.sys[s];
    const int lane = threadIdx.x & 63;
    const int row = sl * 64 + lane;
    const int due = S.snap_mask;
    if (due) {   // run-ahead: x~ of the last iteration, first below these candidates
        for (int t = 0; t < kNumEps; ++t)
            if ((due >> t) & 1) a.snap32[(size_t)t * ((size_t)a.max_slices * 64) + row] = a.x32[row];
    }
    const int mode = S.mode;
    if (mode != kCg32 && mode != kCg64 && mode != kRestart && mode != kResid) return;
    const int len = a.rowlen[row];
    const int64_t base = S.entry0 + a.slice_off[sl] + lane;
    double p;
    if (mode == kCg32) p = cg_product<float, NT>(a, S, a.v32, a.r32, a.dA32, a.dB32, a.q32, base, row, len);
    else if (mode == kCg64) p = cg_product<double, NT>(a, S, a.v64, a.r64, a.dA64, a.dB64, a.q64, base, row, len);
    else p = wave_sum_d(residual<NT>(a, S, mode == kRestart, base, row, len));
    if (lane == 0) a.pslice[2 * (size_t)sl] = p;
}

// Block per system: finish the product's reduction and take its decision.
__global__ void __launch_bounds__(kBlock) k_b_scalar1(BArena a)
{
    __shared__ double sm[kBlock / 64 + 1];
    if ((int)blockIdx.x >= a.step_cnt[1]) return;
    BSys &S = a.sys[a.step_sys[blockIdx.x]];
    const int mode = S.mode;
    if (threadIdx.x == 0 && S.snap_mask) S.snap_mask = 0;   // the product of this step took the copies
    if (mode != kCg32 && mode != kCg64 && mode != kRestart && mode != kResid) return;
    const double v = (mode == kCg32 && a.acc32) ? sys_sum_f(a, S, 0, sm) : sys_sum(a, S, 0, sm);
    if (threadIdx.x != 0) return;
    const double sb = sqrt(S.bb);
    if (mode == kCg32 || mode == kCg64) {
        const double delta = v;
        S.delta = delta;
        if (!isfinite(delta) || !(delta > 0.0)) {
            if (mode == kCg32 && S.auto_eps && !S.eps_set && S.k0_used != 0) {
                // run-ahead: where the FP32 phase stops depends on eps1
                S.ra_stop = kRaBreakdown;
                S.mode = kHold;
                return;
            }
            if (mode == kCg32) {
                S.flags |= MPCG_FLAG_FP32_BREAKDOWN;
                if (S.auto_eps && !S.eps_set && S.k0_used == 0) S.k0_used = S.n1 < S.k0 ? S.n1 : S.k0;
                S.relres_sp = sqrt(S.gamma) / sb;
                S.src = kSrcX32;
                S.ph_it = 0;
                S.mode = kRestart;
            } else {
                S.pend = isfinite(delta) ? MPCG_ENOTSPD : MPCG_ENONFINITE;
                S.mode = kResid;
            }
            return;
        }
        S.alpha = mode == kCg32 ? (double)(float)(S.gamma / delta) : S.gamma / delta;
        S.upd = 1;
    } else if (mode == kRestart) {
        S.gamma = v;
        S.relres_restart = sqrt(v) / sb;
        S.ph_it = 0;
        if (sqrt(v) <= S.thr2) {
            S.mode = kResid;
        } else if (S.n2 >= S.maxit2) {
            S.pend = MPCG_ENOCONV;
            S.mode = kResid;
        } else {
            S.mode = kCg64;
        }
    } else {   // final check
        const double rho = sqrt(v);
        S.relres_final = rho / sb;
        if (S.pend) {
            S.status = S.pend;
            S.mode = kDone;
        } else if (rho <= S.thr2) {
            S.status = MPCG_OK;
            S.mode = kDone;
        } else if (S.restarts < S.max_restarts) {
            S.restarts += 1;
            S.flags |= MPCG_FLAG_FINAL_RESTARTED;
            S.src = kSrcX64;
            S.mode = kRestart;
        } else {
            S.status = MPCG_ENOCONV;
            S.mode = kDone;
        }
    }
}

template <typename T>
__device__ inline double cg_update(const BArena &a, const BSys &S, T *x, T *r, const T *q, const T *dA, const T *dB,
                                   int row)
{
    const T alpha = (T)S.alpha;
    const T *d = (S.ph_it & 1) ? dB : dA;
    x[row] = fma_b<T>(alpha, d[row], x[row]);
    const T rv = fma_b<T>(-alpha, q[row], r[row]);
    r[row] = rv;
    if (sizeof(T) == 4 && a.acc32) return (double)wave_sum_f((float)rv * (float)rv);
    return wave_sum_d((double)rv * (double)rv);
}

__global__ void __launch_bounds__(kBlock) k_b_update(BArena a)
{
    const int k = blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
    if (k >= a.step_cnt[0]) return;
    const int2 e = a.step_map[k];   // slice and its system: no dependent lookup of the owner
    const int sl = e.x, s = e.y;
    if (s < 0) return;
    const BSys &S = a.sys[s];
    if (!S.upd) return;
    const int lane = threadIdx.x & 63;
    const int row = sl * 64 + lane;
    const double p = S.mode == kCg32 ? cg_update<float>(a, S, a.x32, a.r32, a.q32, a.dA32, a.dB32, row)
                                     : cg_update<double>(a, S, a.x64, a.r64, a.q64, a.dA64, a.dB64, row);
    if (lane == 0) a.pslice[2 * (size_t)sl] = p;
}

// Block per system: gamma of the new residual, v ratios, stop tests, beta.
__global__ void __launch_bounds__(kBlock) k_b_scalar2(BArena a)
{
    __shared__ double sm[kBlock / 64 + 1];
    if ((int)blockIdx.x >= a.step_cnt[1]) return;
    BSys &S = a.sys[a.step_sys[blockIdx.x]];
    if (!S.upd) return;
    const double g = (S.mode == kCg32 && a.acc32) ? sys_sum_f(a, S, 0, sm) : sys_sum(a, S, 0, sm);
    if (threadIdx.x != 0) return;
    S.upd = 0;
    const double gp = S.gamma;
    S.gamma_prev = gp;
    S.gamma = g;
    S.ph_it += 1;
    const double sb = sqrt(S.bb);
    if (S.mode == kCg32) {
        S.n1 += 1;
        const bool prefix = S.auto_eps && S.k0_used == 0;
        if (prefix && S.n1 <= S.k0 && S.n1 <= kK0Max) S.ratios[S.n1 - 1] = sqrt(g) / sqrt(gp);
        S.beta = (double)(float)(g / gp);
        if (prefix && (S.n1 >= S.k0 || g == 0.0)) S.k0_used = S.n1;
        if (prefix && S.n1 < S.k0 && g != 0.0) return;   // Algorithm II: k0 iterations first
        if (S.auto_eps && !S.eps_set) {
            // until eps1 is known: record the first crossing of each
            // candidate (x~ is copied by the next product); then either hold
            // (many systems listed: a.hold_above) or run ahead
            const double rg = sqrt(g);
            int due = 0, left = 0;
            for (int t = 0; t < kNumEps; ++t) {
                if (S.cross_iter[t] >= 0) continue;
                if (rg <= S.spec_thr[t]) {
                    S.cross_iter[t] = S.n1;
                    S.cross_gamma[t] = g;
                    due |= 1 << t;
                } else {
                    ++left;
                }
            }
            S.snap_mask = due;
            if (a.step_cnt[1] > a.hold_above) {
                // Until the loosest candidate is crossed every choice of eps1
                // needs these iterations; from the first crossing on they may
                // be wasted, so the system waits there for eps1 without taking
                // bandwidth from the others (no iteration past the chosen
                // eps1, no speculative FP64 phase that the choice may
                // discard).  k_set_eps resumes it from the state the
                // sequential method stops in, as after a run-ahead.
                if (due) {
                    S.ra_stop = left == 0 ? kRaAllCrossed : kRaWait;
                    S.mode = kHold;
                } else if (S.n1 >= S.maxit1) {
                    S.ra_stop = kRaMaxit;
                    S.mode = kHold;
                }
            } else if (left == 0) {
                // every candidate crossed before eps1 is known: the FP64 phase
                // starts now from the tightest candidate's state (x~ of this
                // iteration); k_set_eps keeps it when the chosen candidate
                // crossed at this same iteration, else restarts the FP64 phase
                // from the chosen candidate's copy -- the sequential method's
                // state either way
                S.ra_stop = kRaAllCrossed;
                S.spec = 1;
                S.relres_sp = sqrt(g) / sb;
                S.src = kSrcX32;
                S.ph_it = 0;
                S.mode = kRestart;
            } else if (S.n1 >= S.maxit1) {
                S.ra_stop = kRaMaxit;
                S.mode = kHold;
            }
            return;
        }
        if (sqrt(g) <= S.thr1 || S.n1 >= S.maxit1) {
            if (!(sqrt(g) <= S.thr1)) S.flags |= MPCG_FLAG_FP32_MAXIT;
            S.relres_sp = sqrt(g) / sb;
            S.src = kSrcX32;
            S.ph_it = 0;
            S.mode = kRestart;
        }
    } else {
        S.n2 += 1;
        S.beta = g / gp;
        if (sqrt(g) <= S.thr2) {
            S.mode = kResid;
        } else if (S.n2 >= S.maxit2) {
            S.pend = MPCG_ENOCONV;
            S.mode = kResid;
        }
    }
}

// ----------------------------------------------------------------- 2BFS --

// One block of four waves (a larger block waits longer for room on a CU
// beside the steps).
constexpr int kPlanThreads = 256;

// Single block: retire the level each running system expanded last step
// (appends -> frontier), detect ended sweeps, and list this step's work:
// systems with a frontier that fits in LDS go to the one-block-per-system
// kernel, the others share the multi-block level kernel through an item
// prefix.
__global__ void __launch_bounds__(kPlanThreads) k_bfs_plan(BArena a, int32_t hi_sys, int32_t small_cap)
{
    constexpr int kWaves = kPlanThreads / 64;
    __shared__ int64_t w_items[kWaves];
    __shared__ int32_t w_big[kWaves], w_small[kWaves];
    __shared__ int64_t base_items;
    __shared__ int32_t base_big, base_small;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        base_items = 0;
        base_big = 0;
        base_small = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < hi_sys; c0 += kPlanThreads) {
        const int s = c0 + threadIdx.x;
        int64_t items = 0;
        int big = 0, small = 0;
        if (s < hi_sys) {
            BSys &S = a.sys[s];
            // the fields read, loaded together (one memory latency, not a chain)
            const int mode = S.bfs_mode, c = S.bfs_nxt, lvl = S.bfs_level, sweep = S.bfs_sweep, lanes = S.lanes;
            if (mode == kBfsRun) {
                if (lvl < 0 && sweep == 1) S.ncomp = c;
                if (c == 0) {
                    S.bfs_mode = kBfsSwept;
                } else {
                    S.bfs_nxt = 0;
                    S.bfs_level = lvl + 1;
                    S.bfs_cnt = c;
                    if (c <= small_cap) {
                        small = 1;
                    } else {
                        big = 1;
                        items = (int64_t)c * lanes;
                    }
                }
                S.small = small;
            }
        }
        // exclusive scans of (items, big, small) in system order: inclusive
        // within each wave by shuffles, then the wave totals in order
        int64_t si = items;
        int32_t sb = big, ss = small;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t ti = __shfl_up(si, o, 64);
            const int32_t tb = __shfl_up(sb, o, 64), ts = __shfl_up(ss, o, 64);
            if (lane >= o) {
                si += ti;
                sb += tb;
                ss += ts;
            }
        }
        if (lane == 63) {
            w_items[wid] = si;
            w_big[wid] = sb;
            w_small[wid] = ss;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t ri = base_items;
            int32_t rb = base_big, rs = base_small;
            for (int w = 0; w < kWaves; ++w) {
                const int64_t ti = w_items[w];
                const int32_t tb = w_big[w], ts = w_small[w];
                w_items[w] = ri;
                w_big[w] = rb;
                w_small[w] = rs;
                ri += ti;
                rb += tb;
                rs += ts;
            }
            base_items = ri;
            base_big = rb;
            base_small = rs;
        }
        __syncthreads();
        const int64_t ex_items = w_items[wid] + si - items;
        const int32_t ex_big = w_big[wid] + sb - big, ex_small = w_small[wid] + ss - small;
        if (big) {
            a.act_sys[ex_big] = s;
            a.act_pre[ex_big] = ex_items;
            a.sys[s].item0 = ex_items;
        }
        if (small) a.small_sys[ex_small] = s;
        __syncthreads();   // the wave slots are rewritten by the next chunk
    }
    if (threadIdx.x == 0) {
        a.counts[0] = base_big;
        a.counts[1] = base_small;
        a.items[0] = base_items;
    }
}

// One level of every system on the large list.  Item w belongs to the
// system k with act_pre[k] <= w < act_pre[k + 1]; `lanes` consecutive items
// share a frontier vertex and split its row.
__global__ void __launch_bounds__(kBlock) k_bfs_level_batch(BArena a)
{
    const int nact = a.counts[0];
    if (nact == 0) return;
    const int64_t items = a.items[0];
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t wbase = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); wbase < items; wbase += stride) {
        const int64_t w = wbase + lane;
        int s = -1, u = -1, j = 0, e = 0, lanes = 1, level = 0;
        int64_t base = 0;
        if (w < items) {
            int lo = 0, hi = nact - 1;   // last k with act_pre[k] <= w
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.act_pre[mid] <= w) lo = mid;
                else hi = mid - 1;
            }
            s = a.act_sys[lo];
            const BSys &S = a.sys[s];
            lanes = S.lanes;
            level = S.bfs_level;
            const int64_t loc = w - a.act_pre[lo];
            const int f = (int)(loc >> (__ffs(lanes) - 1)), l = (int)(loc & (lanes - 1));   // lanes: power of two
            const int32_t *qc = (level & 1) ? a.q1 : a.q0;
            u = qc[S.row0 + f];
            if (u >= S.row0 && u < S.row0 + S.n) {
                base = S.entry0 + a.slice_off[u >> 6] + (u & 63);
                j = l;
                e = a.rowlen[u];
            }
        }
        int steps = j < e ? (e - j + lanes - 1) >> (__ffs(lanes) - 1) : 0;
        steps = wave_max_i32(steps);
        for (int t = 0; t < steps; ++t, j += lanes) {   // wave-uniform trip count
            int v = -1;
            bool won = false;
            if (j < e) {
                v = a.col[base + (int64_t)j * 64];
                won = v != u && a.dist[v] < 0 && atomicCAS(&a.dist[v], -1, level + 1) == -1;
            }
            const unsigned long long m = __ballot(won);
            if (m == 0ull) continue;
            // the wave's new vertices of one system take one append: the first
            // winner reserves them all, each winner writes at its rank
            const int l0 = __ffsll(m) - 1;
            const int s0 = __shfl(s, l0, 64);
            if (__all(!won || s == s0)) {
                int pos0 = 0;
                if (lane == l0) pos0 = atomicAdd(&a.sys[s0].bfs_nxt, (int)__popcll(m));
                pos0 = __shfl(pos0, l0, 64);
                if (won) {
                    const int rank = (int)__popcll(m & ((1ull << lane) - 1ull));
                    int32_t *qn = (level & 1) ? a.q0 : a.q1;
                    qn[a.sys[s].row0 + pos0 + rank] = v;
                }
            } else if (won) {   // the wave straddles systems
                BSys &S = a.sys[s];
                const int pos = atomicAdd(&S.bfs_nxt, 1);
                int32_t *qn = (level & 1) ? a.q0 : a.q1;
                qn[S.row0 + pos] = v;
            }
        }
    }
}

// One block per system on the small list: up to max_levels levels with
// the frontier in LDS, each level's result also written to the global queue.
// Leaves the system as the plan expects: bfs_level = last level expanded,
// bfs_nxt = the size of the next frontier (queue (bfs_level + 1) & 1).
// A system of at most kVisBits rows also keeps its visited set in LDS, one
// bit per row: a level then claims a vertex with an LDS atomic and stores
// its distance without waiting, where the other systems claim it with a
// compare-and-swap on dist in HBM.  Either way every vertex is claimed once,
// at its BFS level.  The bits come from the system's copy in HBM when the
// previous launch on it was this kernel (vis_lvl = the level before this
// one), otherwise from dist; the words that changed go back to HBM at exit.
__global__ void __launch_bounds__(kBlock) k_bfs_small_batch(BArena a, int32_t max_levels, int32_t small_cap,
                                                            int64_t max_work)
{
    __shared__ int32_t sq[2][kSmallBfsCap];
    __shared__ __align__(16) uint32_t vis[kVisBits / 32];
    __shared__ int32_t s_cnt, s_lo, s_hi;
    if ((int)blockIdx.x >= a.counts[1]) return;
    const int s = a.small_sys[blockIdx.x];
    BSys &S = a.sys[s];
    const int lanes = S.lanes, row0 = S.row0;
    const int lsh = __ffs(lanes) - 1;   // lanes is a power of two
    const bool lds_vis = S.n <= kVisBits;
    int level = S.bfs_level;
    int cur = S.bfs_cnt;
    {
        const int32_t *qc = (level & 1) ? a.q1 : a.q0;
        for (int i = threadIdx.x; i < cur; i += kBlock) sq[0][i] = qc[row0 + i];
    }
    // words of the system's bits: two per 64-row slice, nw <= kVisBits / 32;
    // rows row0 .. row0 + 32 * nw - 1 are the system's own (padded) rows
    const int nw = ((S.n + 63) >> 6) * 2;
    const bool reuse = lds_vis && S.vis_lvl == level - 1;
    if (lds_vis && reuse) {
        const uint2 *vg = reinterpret_cast<const uint2 *>(a.vis + (row0 >> 5));   // row0 % 64 == 0
        uint2 *vl = reinterpret_cast<uint2 *>(vis);
        for (int p0 = 0; p0 < nw / 2; p0 += 8 * kBlock) {
            uint2 t[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int p = p0 + k * kBlock + (int)threadIdx.x;
                if (p < nw / 2) t[k] = vg[p];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int p = p0 + k * kBlock + (int)threadIdx.x;
                if (p < nw / 2) vl[p] = t[k];
            }
        }
    } else if (lds_vis) {
        // one word per thread from 32 consecutive distances (eight 16-byte loads)
        const int4 *dg = reinterpret_cast<const int4 *>(a.dist + row0);
        for (int w = threadIdx.x; w < nw; w += kBlock) {
            int4 t[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) t[k] = dg[w * 8 + k];
            uint32_t bits = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                bits |= (uint32_t)(t[k].x >= 0) << (4 * k) | (uint32_t)(t[k].y >= 0) << (4 * k + 1) |
                        (uint32_t)(t[k].z >= 0) << (4 * k + 2) | (uint32_t)(t[k].w >= 0) << (4 * k + 3);
            const int r = S.n - w * 32;   // rows of this word inside the system (padding is not visited)
            if (r < 32) bits &= r <= 0 ? 0u : ((1u << r) - 1u);
            vis[w] = bits;
        }
    }
    if (threadIdx.x == 0) {
        s_lo = reuse ? nw : 0;   // empty range [nw, -1] (no overflow in s_lo + tid); a rebuilt set goes back whole
        s_hi = reuse ? -1 : nw - 1;
    }
    int lo = INT32_MAX, hi = -1;
    int c = 0, nxt = 0;
    int64_t work_done = 0;
    for (int rep = 0; rep < max_levels; ++rep) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        int32_t *qn = (level & 1) ? a.q0 : a.q1;
        const int work = cur * lanes;
        for (int w = threadIdx.x; w < work; w += kBlock) {
            const int f = w >> lsh, l = w & (lanes - 1);
            const int u = sq[c][f];
            const int64_t base = S.entry0 + a.slice_off[u >> 6] + (u & 63);
            const int e = a.rowlen[u];
            for (int j = l; j < e; j += lanes) {
                const int v = a.col[base + (int64_t)j * 64];
                if (v == u) continue;
                bool won;
                if (lds_vis) {
                    // admission keeps every column inside [row0, row0 + n)
                    const int lv = v - row0;
                    const uint32_t bit = 1u << (lv & 31);
                    won = !(vis[lv >> 5] & bit) && !(atomicOr(&vis[lv >> 5], bit) & bit);
                    if (won) {
                        a.dist[v] = level + 1;
                        lo = min(lo, lv >> 5);
                        hi = max(hi, lv >> 5);
                    }
                } else {
                    // the compare-and-swap returns the old distance: no read before it
                    // (one dependent memory round trip less per level on a narrow frontier)
                    won = atomicCAS(&a.dist[v], -1, level + 1) == -1;
                }
                if (won) {
                    const int pos = atomicAdd(&s_cnt, 1);
                    if (pos < kSmallBfsCap) sq[c ^ 1][pos] = v;
                    qn[row0 + pos] = v;
                }
            }
        }
        __syncthreads();
        nxt = s_cnt;
        __syncthreads();
        work_done += work;
        if (nxt == 0 || nxt > small_cap || rep + 1 == max_levels || work_done >= max_work) break;
        level += 1;
        cur = nxt;
        c ^= 1;
    }
    if (lds_vis) {
        if (hi >= 0) {
            atomicMin(&s_lo, lo);
            atomicMax(&s_hi, hi);
        }
        __syncthreads();
        // 0 <= s_lo, s_hi < nw: the system's own words
        for (int w = s_lo + (int)threadIdx.x; w <= s_hi; w += kBlock) a.vis[(row0 >> 5) + w] = vis[w];
    }
    if (threadIdx.x == 0) {
        S.bfs_level = level;
        S.bfs_cnt = cur;
        S.bfs_nxt = nxt;
        if (lds_vis) S.vis_lvl = level;
    }
}

// Block j writes the list entries of the chunk's system j: its slot, and the
// slices of its range at their list positions.
__global__ void __launch_bounds__(kBlock) k_worklist(BArena a, ListChunk c)
{
    const int j = blockIdx.x;
    if (c.last && j == 0 && threadIdx.x == 0) {
        a.step_cnt[0] = c.total_slices;
        a.step_cnt[1] = c.total_sys;
    }
    if (j >= c.n) return;
    const int32_t s0 = c.slice0[j], pre = c.pre[j];
    for (int i = threadIdx.x; i < c.nslices[j]; i += kBlock) a.step_map[pre + i] = make_int2(s0 + i, c.slot[j]);
    if (threadIdx.x == 0) a.step_sys[c.first + j] = c.slot[j];
}

void launch_worklist(hipStream_t s, const BArena &a, const ListChunk &c)
{
    hipLaunchKernelGGL(k_worklist, dim3(c.n > 0 ? c.n : 1), dim3(kBlock), 0, s, a, c);
}

// Wave per slice of a split system in a CG phase: d_j = r_j + beta_j d_{j-1}
// (d_0 = r_0), the value the fused product forms per gathered entry, stored
// once for the product to gather (the same fma, so the same bits).
template <typename T>
__device__ inline void dir_rows(const BSys &S, const T *r, T *dA, T *dB, int row)
{
    const int j = S.ph_it;
    T *dnew = (j & 1) ? dB : dA;
    const T *dold = (j & 1) ? dA : dB;
    dnew[row] = j == 0 ? r[row] : fma_b<T>((T)S.beta, dold[row], r[row]);
}

__global__ void __launch_bounds__(kBlock) k_b_dir(BArena a)
{
    const int k = blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
    if (k >= a.step_cnt[0]) return;
    const int2 e = a.step_map[k];
    const int sl = e.x, s = e.y;
    if (s < 0) return;
    const BSys &S = a.sys[s];
    if (!S.split) return;
    const int mode = S.mode;
    const int row = sl * 64 + (threadIdx.x & 63);
    if (mode == kCg32) dir_rows<float>(S, a.r32, a.dA32, a.dB32, row);
    else if (mode == kCg64) dir_rows<double>(S, a.r64, a.dA64, a.dB64, row);
}

void launch_step(hipStream_t s, const BArena &a, int32_t grid_slices, int32_t grid_sys, bool dir)
{
    if (grid_slices <= 0 || grid_sys <= 0) return;
    if (dir) hipLaunchKernelGGL(k_b_dir, dim3(grid_slices), dim3(kBlock), 0, s, a);
    if (a.nt) hipLaunchKernelGGL(k_b_product<true>, dim3(grid_slices), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_b_product<false>, dim3(grid_slices), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_b_scalar1, dim3(grid_sys), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_b_update, dim3(grid_slices), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_b_scalar2, dim3(grid_sys), dim3(kBlock), 0, s, a);
}

void launch_bfs_round(hipStream_t s, const BArena &a, int32_t hi_sys, int small_levels, int small_cap,
                      int64_t small_work, int level_grid)
{
    if (hi_sys <= 0) return;
    hipLaunchKernelGGL(k_bfs_plan, dim3(1), dim3(kPlanThreads), 0, s, a, hi_sys, small_cap);
    hipLaunchKernelGGL(k_bfs_level_batch, dim3(level_grid), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_bfs_small_batch, dim3(hi_sys), dim3(kBlock), 0, s, a, small_levels, small_cap, small_work);
}

// ------------------------------------------------- 2BFS per system (host) --

__global__ void k_b_cc_init(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        a.label[S.row0 + i] = S.row0 + i;   // parent pointers during the hooking
        a.dist[S.row0 + i] = -1;
    }
}

__device__ inline int b_find(int32_t *parent, int x, int *guard)
{
    int p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int steps = 0;
    while (p != x && steps < (1 << 24)) {
        const int pp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (pp != p) __hip_atomic_store(&parent[x], pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = pp;
        ++steps;
    }
    if (steps >= (1 << 24)) *guard = 1;
    return x;
}

// Union-find over the system's edges: roots hooked larger-under-smaller, so
// every component's root is its smallest vertex.
__global__ void __launch_bounds__(kBlock) k_b_cc_hook(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    int guard = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        const int v = S.row0 + i;
        const int64_t base = S.entry0 + a.slice_off[v >> 6] + (v & 63);
        const int e = a.rowlen[v];
        for (int j = 0; j < e; ++j) {
            const int u = a.col[base + (int64_t)j * 64];
            if (u <= v) continue;
            int tries = 0;
            for (;;) {
                int ru = b_find(a.label, u, &guard), rv = b_find(a.label, v, &guard);
                if (ru == rv) break;
                if (ru < rv) { const int t = ru; ru = rv; rv = t; }
                if (atomicCAS(&a.label[ru], ru, rv) == ru) break;
                if (++tries > (1 << 20)) { guard = 1; break; }
            }
        }
    }
    if (guard) atomicOr(&a.sys[sys].bfs_err, kErrGuard);
}

// Labels compressed; roots seed the first sweep at distance 0.
__global__ void __launch_bounds__(kBlock) k_b_cc_seed(BArena a, int32_t sys)
{
    BSys &S = a.sys[sys];
    int guard = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        const int v = S.row0 + i;
        const int r = b_find(a.label, v, &guard);
        a.label[v] = r;   // only v's own entry is rewritten here; finds read roots' entries, which stay put
        if (r == v) {
            a.dist[v] = 0;
            a.best[v] = 0ull;
            const int pos = atomicAdd(&S.bfs_nxt, 1);
            a.q0[S.row0 + pos] = v;
        }
    }
    if (guard) atomicOr(&S.bfs_err, kErrGuard);
}

// First sweep without components: every vertex labelled with vertex 0, which
// seeds the sweep alone (k_b_seed_root, after this kernel).
__global__ void __launch_bounds__(kBlock) k_b_fast_init(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        a.label[S.row0 + i] = S.row0;
        a.dist[S.row0 + i] = -1;
    }
}

__global__ void k_b_seed_root(BArena a, int32_t sys)
{
    if (threadIdx.x != 0) return;
    BSys &S = a.sys[sys];
    a.dist[S.row0] = 0;
    a.best[S.row0] = 0ull;
    a.q0[S.row0] = S.row0;
    S.bfs_nxt = 1;
    S.reached = 0;
}

__global__ void k_b_bfs_arm(BArena a, int32_t sys, int32_t sweep)
{
    if (threadIdx.x == 0) {
        BSys &S = a.sys[sys];
        S.bfs_level = -1;
        S.bfs_sweep = sweep;
        S.vis_lvl = INT32_MIN;   // the stored visited bits belong to an earlier sweep
        S.bfs_mode = kBfsRun;
        S.comp_best = 0ull;
    }
}

__global__ void k_b_zero_nxt(BArena a, int32_t sys)
{
    if (threadIdx.x == 0) a.sys[sys].bfs_nxt = 0;
}

// Per-component farthest vertex of the sweep: key = (dist << 32) | ~v.  A
// connected system sends every vertex to the same key slot, and same-address
// atomics serialise: a wave whose reached vertices share one component takes
// the maximum over its lanes first and issues one atomic.
__global__ void __launch_bounds__(kBlock) k_b_argmax(BArena a, int32_t sys, int32_t count)
{
    BSys &S = a.sys[sys];
    const int lane = threadIdx.x & 63;
    // wave-uniform loop: every lane of a wave walks the same bases
    for (int base = blockIdx.x * kBlock + (threadIdx.x & ~63); base < S.n; base += gridDim.x * kBlock) {
        const int i = base + lane;
        int lab = -1;
        unsigned long long key = 0ull;
        if (i < S.n) {
            const int v = S.row0 + i;
            const int d = a.dist[v];
            if (d >= 0) {
                key = ((unsigned long long)(unsigned)d << 32) | (unsigned long long)(0xffffffffu - (unsigned)v);
                lab = a.label[v];
            }
        }
        const unsigned long long m = __ballot(lab >= 0);
        if (m == 0ull) continue;
        if (count && lane == 0) atomicAdd(&S.reached, (int)__popcll(m));   // the first sweep's reach
        const int l0 = __ffsll((unsigned long long)m) - 1;
        const int L = __shfl(lab, l0, 64);
        if (__all(lab < 0 || lab == L)) {
            unsigned long long kmax = key;   // lanes without a vertex hold 0, below every key
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(kmax, off, 64);
                kmax = kmax > o ? kmax : o;
            }
            if (lane == l0) atomicMax(&a.best[L], kmax);
        } else if (lab >= 0) {
            atomicMax(&a.best[lab], key);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_b_fill_dist(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) a.dist[S.row0 + i] = -1;
}

// Second sweep from t_c of every component c.
__global__ void __launch_bounds__(kBlock) k_b_seed_far(BArena a, int32_t sys)
{
    BSys &S = a.sys[sys];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        const int v = S.row0 + i;
        if (a.label[v] != v) continue;
        const int t = (int)(0xffffffffu - (unsigned)(a.best[v] & 0xffffffffull));
        if (t < S.row0 || t >= S.row0 + S.n) continue;   // cannot happen: the root itself has a key
        a.tarr[v] = t;
        a.best[v] = 0ull;
        a.dist[t] = 0;
        const int pos = atomicAdd(&S.bfs_nxt, 1);
        a.q0[S.row0 + pos] = t;
    }
}

// Best component: largest eccentricity, first (smallest root) on ties.
__global__ void __launch_bounds__(kBlock) k_b_comp_best(BArena a, int32_t sys)
{
    BSys &S = a.sys[sys];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < S.n; i += gridDim.x * kBlock) {
        const int c = S.row0 + i;
        if (a.label[c] != c) continue;
        const unsigned long long ecc = a.best[c] >> 32;
        atomicMax(&S.comp_best, (ecc << 32) | (unsigned long long)(0xffffffffu - (unsigned)c));
    }
}

__global__ void k_b_feat_final(BArena a, int32_t sys)
{
    if (threadIdx.x != 0) return;
    BSys &S = a.sys[sys];
    const unsigned long long key = S.comp_best;
    const int comp = (int)(0xffffffffu - (unsigned)(key & 0xffffffffull));
    if (key == 0ull || comp < S.row0 || comp >= S.row0 + S.n) {
        S.bfs_err |= kErrGuard;
        S.bfs_mode = kBfsDone;
        return;
    }
    S.pdiam = (int)(key >> 32);
    S.bfs_t = a.tarr[comp] - S.row0;
    S.bfs_u = (int)(0xffffffffu - (unsigned)(a.best[comp] & 0xffffffffull)) - S.row0;
    S.bfs_mode = kBfsDone;
}

static int rows_grid(int n)
{
    int g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    return g < 1 ? 1 : g;
}

// the kernels walk the system's rows grid-stride: the grid follows its size
void launch_bfs_start(hipStream_t s, const BArena &a, int32_t sys, int32_t n)
{
    const int g = rows_grid(n);
    hipLaunchKernelGGL(k_b_zero_nxt, dim3(1), dim3(64), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_cc_init, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_cc_hook, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_cc_seed, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_bfs_arm, dim3(1), dim3(64), 0, s, a, sys, 1);
}

void launch_bfs_fast_start(hipStream_t s, const BArena &a, int32_t sys, int32_t n)
{
    const int g = rows_grid(n);
    hipLaunchKernelGGL(k_b_fast_init, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_seed_root, dim3(1), dim3(64), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_bfs_arm, dim3(1), dim3(64), 0, s, a, sys, 1);
}

void launch_bfs_next_sweep(hipStream_t s, const BArena &a, int32_t sys, int32_t n)
{
    const int g = rows_grid(n);
    hipLaunchKernelGGL(k_b_argmax, dim3(g), dim3(kBlock), 0, s, a, sys, 1);
    hipLaunchKernelGGL(k_b_fill_dist, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_zero_nxt, dim3(1), dim3(64), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_seed_far, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_bfs_arm, dim3(1), dim3(64), 0, s, a, sys, 2);
}

void launch_bfs_finish(hipStream_t s, const BArena &a, int32_t sys, int32_t n)
{
    const int g = rows_grid(n);
    hipLaunchKernelGGL(k_b_argmax, dim3(g), dim3(kBlock), 0, s, a, sys, 0);
    hipLaunchKernelGGL(k_b_comp_best, dim3(g), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_b_feat_final, dim3(1), dim3(64), 0, s, a, sys);
}

// ------------------------------------------------------------ band 2BFS --
//
// A system whose entries all lie within |i - j| <= 31 has, for every offset
// d = j - i present, a bit vector over its rows: bit v of word d says that
// row v - d has an entry at offset d, i.e. the edge (v - d) -> v.  One level
// of a sweep is then, for every 32-row word of the window, the OR over the
// offsets of (that vector AND the frontier shifted by d), minus the visited
// rows: each row of the next level is found from the rows that list it,
// exactly the vertices a level that expands the frontier's rows finds.  A
// wave keeps 64 words (2,048 rows) of the frontier in registers, one per
// lane, and the words of the offsets' vectors for the same rows in LDS; the
// window moves with the frontier.  The frontier of a band moves by at most
// one word per level, so a level touches only the window; a frontier wider
// than 62 words (it cannot occur on a band swept from one end) ends the
// attempt and the system takes the level kernels.

// The system's words of dm are ORed into below: zero them first.
__global__ void __launch_bounds__(kBlock) k_band_clear(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    const int64_t words = (int64_t)((S.n + 31) >> 5) * 64;
    uint32_t *dw = a.dm + (size_t)(S.row0 >> 5) * 64;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlock)
        dw[i] = 0u;
}

// Wave per slice: for each offset d present, the slice's rows that have an
// entry at d (a ballot) mark rows u + d of dm's word d, i.e. 64 bits placed
// at row 64 j + d, across up to three words.
__global__ void __launch_bounds__(kBlock) k_band_masks(BArena a, int32_t sys)
{
    const BSys &S = a.sys[sys];
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
    if (j >= S.nslices) return;
    const int sl = S.slice0 + j;
    const int g = S.row0 + j * 64 + lane;
    const int len = a.rowlen[g];
    const int64_t base = S.entry0 + a.slice_off[sl] + lane;
    unsigned long long om = 0ull;
    for (int k = 0; k < len; ++k) {
        const int d = a.col[base + (int64_t)k * 64] - g;
        if (d != 0 && d >= -kBandMaxBw && d <= kBandMaxBw) om |= 1ull << (d + 32);
    }
    const int nw = (S.n + 31) >> 5;
    uint32_t *dw = a.dm + (size_t)(S.row0 >> 5) * 64;
    unsigned long long pres = S.doffs;   // the same in every lane: a wave-uniform loop
    while (pres) {
        const int k = __ffsll(pres) - 1;
        pres &= pres - 1ull;
        const unsigned long long b = __ballot((om >> k) & 1ull);
        if (b == 0ull) continue;
        const int d = k - 32;
        const int first = 64 * j + d;                   // local row of bit 0 (may be negative)
        const int w0 = first >= 0 ? first >> 5 : -((31 - first) >> 5);   // floor(first / 32)
        const int sh = first - 32 * w0;                 // 0..31
        const unsigned long long lo = b << sh;
        if (lane < 3) {
            const uint32_t part = lane == 0 ? (uint32_t)lo
                                  : lane == 1 ? (uint32_t)(lo >> 32)
                                              : (sh ? (uint32_t)(b >> (64 - sh)) : 0u);
            const int w = w0 + lane;
            if (part && w >= 0 && w < nw) atomicOr(&dw[(size_t)w * 64 + k], part);
        }
    }
}

// The offsets' words of one window position, in registers: lane l holds
// word W0 + l of every listed offset (zero outside the system).  Offsets
// d < 0 first (slots 1..31 of the offset mask), then d > 0 (slots 33..63).
template <int NH>
struct BandOffs {
    int nneg, npos;
    int sneg[NH], spos[NH];           // dm slots
    uint32_t mneg[NH], mpos[NH];      // the window's words
};

template <int NH>
__device__ inline void band_load(const uint32_t *dw, int W0, int nw, BandOffs<NH> &o)
{
    const int w = W0 + (int)threadIdx.x;
    const bool in = w >= 0 && w < nw;
    const uint32_t *p = dw + (size_t)(in ? w : 0) * 64;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        o.mneg[k] = (in && k < o.nneg) ? p[o.sneg[k]] : 0u;
        o.mpos[k] = (in && k < o.npos) ? p[o.spos[k]] : 0u;
    }
}

// V: the system's visited bits in HBM, touched only when the window moves
// (the window's words live in a register per lane).  Another lane may have
// written a word earlier: agent-scope accesses (no stale L1 line) after a
// wait for this wave's stores.
__device__ inline uint32_t band_vload(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void band_vstore(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One sweep from local row src.  Returns false when the frontier outgrows
// the window; else ecc (the last level), far (its smallest row) and reached.
template <int NH>
__device__ inline bool band_sweep(const uint32_t *dw, int n, int nw, BandOffs<NH> &o, uint32_t *V, int src,
                                  int &ecc, int &far, int &reached)
{
    const int lane = threadIdx.x;
    for (int w = lane; w < nw; w += 64) band_vstore(&V[w], 0u);
    __threadfence_block();
    int W0 = (src >> 5) - 31;
    band_load<NH>(dw, W0, nw, o);
    uint32_t F = lane == 31 ? (1u << (src & 31)) : 0u;
    int w = W0 + lane;
    uint32_t Vr = (w >= 0 && w < nw) ? F : 0xffffffffu;   // rows outside the system count as visited
    ecc = 0;
    far = src;
    int cnt = lane == 31 ? 1 : 0;
    bool ok = true;
    for (int lev = 0; lev < n; ++lev) {   // every level reaches a new row: at most n - 1 of them
        const uint32_t up = __shfl_up(F, 1, 64), dn = __shfl_down(F, 1, 64);
        const uint32_t fp = lane == 0 ? 0u : up, fn = lane == 63 ? 0u : dn;
        // bit b of a term: frontier row 32 (W0 + lane) + b - d, for the rows listed under d
        // (the words of unlisted k are zero: no branch per offset)
        uint32_t acc = 0u;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            acc |= __builtin_amdgcn_alignbit(fn, F, 32 - o.sneg[k]) & o.mneg[k];   // -d = 32 - slot
            acc |= __builtin_amdgcn_alignbit(F, fp, 64 - o.spos[k]) & o.mpos[k];   // 32 - d
        }
        const uint32_t nv = acc & ~Vr;
        const unsigned long long any = __ballot(nv != 0u);
        if (any == 0ull) break;
        Vr |= nv;
        F = nv;
        ++ecc;
        cnt += __popc(nv);
        const int lo = __ffsll(any) - 1, hi = 63 - __clzll(any);
        const uint32_t nlo = __builtin_amdgcn_readlane(nv, lo);
        far = (W0 + lo) * 32 + __ffs(nlo) - 1;
        if (lo == 0 || hi == 63) {
            if (hi - lo > 61) {
                ok = false;
                break;
            }
            if (w >= 0 && w < nw) band_vstore(&V[w], Vr);
            // moving up: the frontier's first word to lane 1; down: its last to lane 62
            const int W0n = hi == 63 ? W0 + lo - 1 : W0 + hi - 62;
            const int from = lane + (W0n - W0);
            const uint32_t Fs = __shfl(F, from & 63, 64);
            F = (from >= 0 && from < 64) ? Fs : 0u;
            W0 = W0n;
            w = W0 + lane;
            __threadfence_block();
            Vr = (w >= 0 && w < nw) ? band_vload(&V[w]) : 0xffffffffu;
            band_load<NH>(dw, W0, nw, o);
        }
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) cnt += __shfl_xor(cnt, o2, 64);
    reached = cnt;
    return ok;
}

// One wave per listed system: both sweeps (from row 0, then from the first
// sweep's far row), the result in the system's BFS fields.  NH: the most
// offsets of one sign the launch's systems have.
template <int NH>
__global__ void __launch_bounds__(64) k_bfs_band(BArena a, BandList L)
{
    if ((int)blockIdx.x >= L.cnt) return;
    BSys &S = a.sys[L.slot[blockIdx.x]];
    const int lane = threadIdx.x;
    const int n = S.n, nw = (n + 31) >> 5;
    const unsigned long long pres = S.doffs;
    BandOffs<NH> o;
    {
        unsigned long long mn = pres & 0xffffffffull, mp = pres >> 33;   // slots 1..31; 33..63 (d = 1..31)
        o.nneg = __popcll(mn);
        o.npos = __popcll(mp);
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            o.sneg[k] = mn ? __ffsll(mn) - 1 : 0;
            mn &= mn - 1ull;
            o.spos[k] = mp ? __ffsll(mp) + 32 : 0;
            mp &= mp - 1ull;
        }
    }
    const uint32_t *dw = a.dm + (size_t)(S.row0 >> 5) * 64;
    uint32_t *V = a.vis + (S.row0 >> 5);
    int ecc1 = 0, t = 0, reached = 0, ecc2 = 0, u = 0, r2 = 0;
    int fail = 0;
    if (o.nneg > NH || o.npos > NH) fail = 1;   // the launch's unrolling does not cover it (host error)
    else if (!band_sweep<NH>(dw, n, nw, o, V, 0, ecc1, t, reached)) fail = 1;
    else if (reached != n) fail = 2;
    else if (!band_sweep<NH>(dw, n, nw, o, V, t, ecc2, u, r2)) fail = 1;
    if (lane == 0) {
        S.band_fail = fail;
        S.reached = reached;
        if (!fail) {
            S.pdiam = ecc2;
            S.bfs_t = t;
            S.bfs_u = u;
            S.ncomp = 1;
            S.bfs_mode = kBfsDone;
        }
    }
}

void launch_band_masks(hipStream_t s, const BArena &a, int32_t sys, int32_t nslices)
{
    hipLaunchKernelGGL(k_band_clear, dim3(rows_grid(nslices * 64)), dim3(kBlock), 0, s, a, sys);
    hipLaunchKernelGGL(k_band_masks, dim3((nslices + kSlicesPerBlock - 1) / kSlicesPerBlock), dim3(kBlock), 0, s,
                       a, sys);
}

void launch_bfs_band(hipStream_t s, const BArena &a, const BandList &l)
{
    if (l.cnt <= 0) return;
    if (l.nh_max <= 4) hipLaunchKernelGGL(k_bfs_band<4>, dim3(l.cnt), dim3(64), 0, s, a, l);
    else if (l.nh_max <= 8) hipLaunchKernelGGL(k_bfs_band<8>, dim3(l.cnt), dim3(64), 0, s, a, l);
    else if (l.nh_max <= 16) hipLaunchKernelGGL(k_bfs_band<16>, dim3(l.cnt), dim3(64), 0, s, a, l);
    else hipLaunchKernelGGL(k_bfs_band<31>, dim3(l.cnt), dim3(64), 0, s, a, l);
}

// ------------------------------------------------------- admission (host) --

static int adm_grid(const AdmitList &l, int spb)
{
    int g = 0;
    for (int j = 0; j < l.cnt; ++j) g += (l.nsl[j] + spb - 1) / spb;
    return g;
}

void launch_admit_stage1(hipStream_t s, const BArena &a, const AdmitList &l)
{
    if (l.cnt <= 0) return;
    hipLaunchKernelGGL(k_admit_fill_l, dim3(adm_grid(l, kBlock)), dim3(kBlock), 0, s, a, l);
    hipLaunchKernelGGL(k_admit_rows_l, dim3(adm_grid(l, kSlicesPerBlock)), dim3(kBlock), 0, s, a, l);
    hipLaunchKernelGGL(k_admit_scan_l, dim3(l.cnt), dim3(1024), 0, s, a, l);
}

void launch_admit_stage2(hipStream_t s, const BArena &a, const AdmitList &l)
{
    if (l.cnt <= 0) return;
    hipLaunchKernelGGL(k_admit_entries_l, dim3(adm_grid(l, kSlicesPerBlock)), dim3(kBlock), 0, s, a, l);
    hipLaunchKernelGGL(k_admit_finish_l, dim3(l.cnt), dim3(kBlock), 0, s, a, l);
    hipLaunchKernelGGL(k_admit_publish_l, dim3(adm_grid(l, kBlock)), dim3(kBlock), 0, s, a, l);
}

void launch_release(hipStream_t s, const BArena &a, int32_t sys, int32_t slice0, int32_t nslices)
{
    hipLaunchKernelGGL(k_release, dim3(rows_grid(nslices)), dim3(kBlock), 0, s, a, sys, slice0, nslices);
}

void launch_cancel(hipStream_t s, const BArena &a, int32_t sys)
{
    hipLaunchKernelGGL(k_cancel, dim3(1), dim3(64), 0, s, a, sys);
}

void launch_bfs_cancel(hipStream_t s, const BArena &a, int32_t sys)
{
    hipLaunchKernelGGL(k_bfs_cancel, dim3(1), dim3(64), 0, s, a, sys);
}

void launch_set_eps(hipStream_t s, const BArena &a, int32_t sys, double eps1, int32_t ci)
{
    hipLaunchKernelGGL(k_set_eps, dim3(1), dim3(64), 0, s, a, sys, eps1, ci);
}

}  // namespace batch
}  // namespace mpcg
