// CG kernels for gfx950: CSR ingest/cast, CSR-stream SpMV with per-row fma
// chains, fused axpy + dot updates, and a single-pass deterministic grid
// reduction that finalises the CG scalars on the device.
//
// One CG iteration is two launches:
//   k_spmv<CG>   d_i = r_i + beta_i d_{i-1} (own rows written, gathered
//                columns recomputed on the fly), q = A d_i, delta = d_i.q,
//                last block: alpha = gamma / delta (rounded to the working
//                precision), breakdown test.
//   k_update     x += alpha d_i, r -= alpha q, gamma' = r.r, last block:
//                beta = gamma'/gamma, decay ratio for v (eq. 13), stop test.
// These are the steps of the CG procedure in the paper's "Conjugate Gradient
// Method" section with the direction update moved to the start of the next
// product; the arithmetic of each element is unchanged.

#include "mpcg_internal.hpp"

#include <cmath>

namespace mpcg {

// ------------------------------------------------------------ helpers --

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum (kBlock threads): butterfly inside each wave, then
// wave 0..3 in order.  Valid in thread 0.
__device__ inline double block_sum(double v, double *sm)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kBlock / 64; ++i) s += sm[i];
    }
    __syncthreads();
    return s;
}

__device__ inline void store_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_agent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single-pass grid reduction of NV doubles.  Every block calls it exactly
// once; it returns true in the last block to arrive, where out[] (thread 0)
// holds the sums taken in block order 0..nblk-1 (same order every run).
template <int NV>
__device__ bool grid_reduce(const double (&v)[NV], double *part, uint32_t *ticket, int nblk,
                            int bid, double (&out)[NV])
{
    __shared__ double sm[kBlock / 64];
    __shared__ int amlast;
    double bs[NV];
    for (int j = 0; j < NV; ++j) bs[j] = block_sum(v[j], sm);
    if (threadIdx.x == 0) {
        for (int j = 0; j < NV; ++j) store_agent(part + (size_t)bid * NV + j, bs[j]);
        __threadfence();
        uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        amlast = (t == (uint32_t)(nblk - 1));
    }
    __syncthreads();
    if (!amlast) return false;
    __threadfence();
    for (int j = 0; j < NV; ++j) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nblk; i += kBlock) acc += load_agent(part + (size_t)i * NV + j);
        out[j] = block_sum(acc, sm);
    }
    if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Blocks are dispatched round-robin over the XCDs; map them so that each XCD
// walks a contiguous range of rows and its own L2 sees the x-gather reuse.
__device__ inline int xcd_remap(int b, int nb)
{
    const int q = nb / kNumXcd, rem = nb % kNumXcd;
    const int x = b % kNumXcd, i = b / kNumXcd;
    return x * q + (x < rem ? x : rem) + i;
}

template <typename T> __device__ inline T fmaT(T a, T b, T c);
template <> __device__ inline float fmaT<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ inline double fmaT<double>(double a, double b, double c) { return fma(a, b, c); }

// --------------------------------------------------------------- ingest --

__global__ void __launch_bounds__(kBlock)
k_ingest(const void *rp_in, int rp_is_i64, const int32_t *__restrict__ col,
         const double *__restrict__ val, const double *__restrict__ b, int32_t n, int64_t nnz,
         int32_t *__restrict__ rp32_out, float *__restrict__ val32_out, DevState *st)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int err = 0, len = 0;
    if (i < n) {
        int64_t lo, hi;
        if (rp_is_i64) {
            lo = ((const int64_t *)rp_in)[i];
            hi = ((const int64_t *)rp_in)[i + 1];
        } else {
            lo = ((const int32_t *)rp_in)[i];
            hi = ((const int32_t *)rp_in)[i + 1];
        }
        if (i == 0 && lo != 0) err |= kErrRowPtr;
        if (i == n - 1 && hi != nnz) err |= kErrRowPtr;
        if (lo < 0 || hi < lo || hi > nnz) {
            err |= kErrRowPtr;
        } else {
            len = (int)(hi - lo);
            int prev = -1;
            for (int64_t k = lo; k < hi; ++k) {
                const int c = col[k];
                if (c < 0 || c >= n) err |= kErrCol;
                if (c <= prev) err |= kErrUnsorted;
                prev = c;
                const double v = val[k];
                if (!isfinite(v)) err |= kErrNonFiniteA;
                if (val32_out) val32_out[k] = (float)v;
            }
        }
        if (rp32_out) {
            rp32_out[i] = (int32_t)lo;
            if (i == n - 1) rp32_out[n] = (int32_t)hi;
        }
        if (b && !isfinite(b[i])) err |= kErrNonFiniteB;
    }
    // one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        err |= __shfl_xor(err, off, 64);
        const int o = __shfl_xor(len, off, 64);
        len = len > o ? len : o;
    }
    if ((threadIdx.x & 63) == 0) {
        if (err) atomicOr(&st->ing_err, err);
        atomicMax(&st->max_row, len);
    }
}

void launch_ingest(hipStream_t s, const void *rp_in, int rp_is_i64, const int32_t *col,
                   const double *val, const double *b, int32_t n, int64_t nnz, int32_t *rp32_out,
                   float *val32_out, DevState *st)
{
    const int grid = (int)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ingest, dim3(grid), dim3(kBlock), 0, s, rp_in, rp_is_i64, col, val, b, n,
                       nnz, rp32_out, val32_out, st);
}

// ---------------------------------------------------------------- fills --

__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}
__global__ void k_fill_f32(float *p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

static int fill_grid(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_fill_f64(hipStream_t s, double *p, int64_t n, double v)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n, v);
}
void launch_fill_f32(hipStream_t s, float *p, int64_t n, float v)
{
    hipLaunchKernelGGL(k_fill_f32, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n, v);
}
void launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, n, v);
}

// ------------------------------------------------------------ phase init --

// Sets the stop test of a phase from the freshly reduced gamma.
__device__ inline void start_phase(DevState *st, double gamma, double eps, int abs_tol, int32_t maxit)
{
    st->gamma = gamma;
    st->beta = 0.0;
    st->thr = abs_tol ? eps : eps * sqrt(st->bnorm2);
    st->maxit = maxit;
    if (sqrt(gamma) <= st->thr) {
        st->live = 0; st->reason = kConverged;
    } else if (st->iter >= maxit) {
        st->live = 0; st->reason = kMaxit;
    } else {
        st->live = 1; st->reason = kRunning;
    }
}

// FP32 phase from x~ = 0: r~ = float32(b), old direction = 0,
// gamma = r~.r~ and ||b||^2, both accumulated in FP64.
__global__ void __launch_bounds__(kBlock)
k_init32(const double *__restrict__ b, float *__restrict__ x, float *__restrict__ r,
         float *__restrict__ dA, int32_t n, double eps, int abs_tol, int32_t maxit, int32_t k0rec,
         double *part, DevState *st)
{
    double s[2] = {0.0, 0.0};
    const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kVecPerThread; ++j) {
        const int64_t i = base + j * kBlock;
        if (i < n) {
            const double bv = b[i];
            const float rv = (float)bv;
            r[i] = rv;
            x[i] = 0.0f;
            dA[i] = 0.0f;
            s[0] = fma((double)rv, (double)rv, s[0]);
            s[1] = fma(bv, bv, s[1]);
        }
    }
    double out[2];
    if (grid_reduce<2>(s, part, &st->tk_init, gridDim.x, blockIdx.x, out) && threadIdx.x == 0) {
        st->bnorm2 = out[1];
        st->iter = 0;
        st->k0rec = k0rec;
        start_phase(st, out[0], eps, abs_tol, maxit);
    }
}

void launch_init32(hipStream_t s, const double *b, float *x, float *r, float *dA, int32_t n,
                   double eps, int abs_tol, int32_t maxit, int32_t k0rec, double *part, DevState *st)
{
    const int grid = (n + kVecTile - 1) / kVecTile;
    hipLaunchKernelGGL(k_init32, dim3(grid), dim3(kBlock), 0, s, b, x, r, dA, n, eps, abs_tol, maxit,
                       k0rec, part, st);
}
// Continue a phase with a new stop test (Algorithm II after the k0 prefix).
__global__ void k_set_phase(DevState *st, double thr, int32_t maxit, int32_t k0rec, int32_t reset_iter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (reset_iter) st->iter = 0;
        st->thr = thr;
        st->maxit = maxit;
        st->k0rec = k0rec;
        if (sqrt(st->gamma) <= thr) {
            st->live = 0; st->reason = kConverged;
        } else if (st->iter >= maxit) {
            st->live = 0; st->reason = kMaxit;
        } else {
            st->live = 1; st->reason = kRunning;
        }
    }
}

// Measurement set-up: a live recurrence that no test can stop.
__global__ void k_timing_state(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->gamma = 1.0;
        st->alpha = 1e-3;
        st->beta = 0.5;
        st->thr = 0.0;
        st->iter = 0;
        st->maxit = 0x7fffffff;
        st->k0rec = 0;
        st->live = 1;
        st->reason = kRunning;
    }
}

void launch_timing_state(hipStream_t s, DevState *st)
{
    hipLaunchKernelGGL(k_timing_state, dim3(1), dim3(64), 0, s, st);
}

void launch_set_phase(hipStream_t s, DevState *st, double thr, int32_t maxit, int32_t k0rec,
                      int32_t reset_iter)
{
    hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, st, thr, maxit, k0rec, reset_iter);
}

// ------------------------------------------------------------- CSR-stream --

enum SpmvMode { kModeCg = 0, kModeRestart = 1, kModeResid = 2, kModePlain = 3 };

template <typename T>
struct SpmvArgs {
    const int32_t *rp;
    const int32_t *col;
    const T *val;
    int32_t n;
    int32_t R;        // rows per block
    // CG
    const T *r;
    T *dA, *dB, *q;
    // restart / residual (T = double)
    const float *x32;
    const double *x64in;
    double *x64out;
    const double *b;
    double *rout;
    double *dzA, *dzB;
    double eps;
    int32_t abs_tol, maxit;
    // plain
    const T *xin;
    T *yout;
    double *part;
    DevState *st;
};

// A block owns R consecutive rows.  Phase 1 streams the block's entries
// [rp[row0], rp[row1]) in LDS-sized chunks with coalesced col/val loads and
// gathers the vector entry of each column; phase 2 lets thread t run the fma
// chain of row row0 + t over its entries in CSR order, starting from 0 -- the
// same rounding sequence as a sequential row loop.
template <int MODE, typename T>
__global__ void __launch_bounds__(kBlock) k_spmv(SpmvArgs<T> a)
{
    constexpr int CHUNK = kLdsBytes / (2 * (int)sizeof(T));
    __shared__ T s_val[CHUNK];
    __shared__ T s_x[CHUNK];
    DevState *st = a.st;
    if (MODE == kModeCg) {
        if (!st->live) return;
    }
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    const int row0 = bid * a.R;
    const int row1 = min(row0 + a.R, a.n);

    T beta = T(0);
    const T *dold = nullptr;
    T *dnew = nullptr;
    if (MODE == kModeCg) {
        const int it = st->iter;
        beta = (T)st->beta;
        dold = (it & 1) ? a.dB : a.dA;
        dnew = (it & 1) ? a.dA : a.dB;
    }

    const int my_row = row0 + tid;
    const bool has = (tid < a.R) && (my_row < row1);
    int my_lo = 0, my_hi = 0;
    if (has) {
        my_lo = a.rp[my_row];
        my_hi = a.rp[my_row + 1];
    }
    const int lo = a.rp[row0];
    const int hi = a.rp[row1];

    T acc = T(0);
    for (int c0 = lo; c0 < hi; c0 += CHUNK) {
        const int cn = min(CHUNK, hi - c0);
        for (int j = tid; j < cn; j += kBlock) {
            const int k = c0 + j;
            const int c = a.col[k];
            s_val[j] = a.val[k];
            T g;
            if (MODE == kModeCg) {
                g = fmaT<T>(beta, dold[c], a.r[c]);
            } else if (MODE == kModeRestart || MODE == kModeResid) {
                g = a.x32 ? (T)a.x32[c] : (T)a.x64in[c];
            } else {
                g = a.xin[c];
            }
            s_x[j] = g;
        }
        __syncthreads();
        if (has) {
            const int kb = max(my_lo, c0), ke = min(my_hi, c0 + cn);
            for (int k = kb; k < ke; ++k) acc = fmaT<T>(s_val[k - c0], s_x[k - c0], acc);
        }
        __syncthreads();
    }

    if (MODE == kModePlain) {
        if (has) a.yout[my_row] = acc;
        return;
    }

    // restart also reduces ||b||^2, so that FP64-only runs (x = 0) and mixed
    // runs share one reduction layout for gamma and for the stop threshold
    constexpr int NV = (MODE == kModeRestart) ? 2 : 1;
    double s[NV];
    for (int j = 0; j < NV; ++j) s[j] = 0.0;
    if (has) {
        if (MODE == kModeCg) {
            const T dn = fmaT<T>(beta, dold[my_row], a.r[my_row]);
            dnew[my_row] = dn;
            a.q[my_row] = acc;
            s[0] = fma((double)dn, (double)acc, 0.0);
        } else {
            const double bv = a.b[my_row];
            const double res = bv - (double)acc;
            if (MODE == kModeRestart) {
                if (a.x32) a.x64out[my_row] = (double)a.x32[my_row];
                a.rout[my_row] = res;
                const int it = st->iter;
                double *dz = (it & 1) ? a.dzB : a.dzA;
                dz[my_row] = 0.0;
                s[NV - 1] = fma(bv, bv, 0.0);
            }
            s[0] = fma(res, res, 0.0);
        }
    }
    double out[NV];
    uint32_t *tk = (MODE == kModeCg) ? &st->tk_spmv : &st->tk_misc;
    if (grid_reduce<NV>(s, a.part, tk, gridDim.x, bid, out) && threadIdx.x == 0) {
        const double sum = out[0];
        if (MODE == kModeCg) {
            st->delta = sum;
            if (!isfinite(sum)) {
                st->live = 0; st->reason = kNonFinite;
            } else if (!(sum > 0.0)) {
                st->live = 0; st->reason = kNotSpd;
            } else {
                st->alpha = (double)(T)(st->gamma / sum);
            }
        } else if (MODE == kModeRestart) {
            st->bnorm2 = out[NV - 1];
            start_phase(st, sum, a.eps, a.abs_tol, a.maxit);
        } else {
            st->resid2 = sum;
        }
    }
}

template <typename T>
static int spmv_grid(int32_t n, int R)
{
    return (n + R - 1) / R;
}

template <typename T>
void launch_cg_spmv(hipStream_t s, const int32_t *rp, const int32_t *col, const T *val, int32_t n,
                    int R, const T *r, T *dA, T *dB, T *q, double *part, DevState *st)
{
    SpmvArgs<T> a{};
    a.rp = rp; a.col = col; a.val = val; a.n = n; a.R = R;
    a.r = r; a.dA = dA; a.dB = dB; a.q = q; a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeCg, T>), dim3(spmv_grid<T>(n, R)), dim3(kBlock), 0, s, a);
}

void launch_restart(hipStream_t s, const int32_t *rp, const int32_t *col, const double *val,
                    int32_t n, int R, const float *x32, double *x64, const double *b, double *r,
                    double *dA, double *dB, double eps, int abs_tol, int32_t maxit, double *part,
                    DevState *st)
{
    SpmvArgs<double> a{};
    a.rp = rp; a.col = col; a.val = val; a.n = n; a.R = R;
    a.x32 = x32; a.x64in = x64; a.x64out = x64; a.b = b; a.rout = r; a.dzA = dA; a.dzB = dB;
    a.eps = eps; a.abs_tol = abs_tol; a.maxit = maxit; a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeRestart, double>), dim3(spmv_grid<double>(n, R)), dim3(kBlock), 0,
                       s, a);
}

void launch_resid(hipStream_t s, const int32_t *rp, const int32_t *col, const double *val,
                  int32_t n, int R, const double *x64, const double *b, double *part, DevState *st)
{
    SpmvArgs<double> a{};
    a.rp = rp; a.col = col; a.val = val; a.n = n; a.R = R;
    a.x32 = nullptr; a.x64in = x64; a.b = b; a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeResid, double>), dim3(spmv_grid<double>(n, R)), dim3(kBlock), 0,
                       s, a);
}

template <typename T>
void launch_spmv_plain(hipStream_t s, const int32_t *rp, const int32_t *col, const T *val,
                       int32_t n, int R, const T *x, T *y)
{
    SpmvArgs<T> a{};
    a.rp = rp; a.col = col; a.val = val; a.n = n; a.R = R; a.xin = x; a.yout = y;
    hipLaunchKernelGGL((k_spmv<kModePlain, T>), dim3(spmv_grid<T>(n, R)), dim3(kBlock), 0, s, a);
}

// ------------------------------------------------------------- update --

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_update(int32_t n, T *__restrict__ x, T *__restrict__ r, const T *__restrict__ q,
         const T *__restrict__ dA, const T *__restrict__ dB, double *part, DevState *st)
{
    if (!st->live) return;
    const int it = st->iter;
    const T alpha = (T)st->alpha;
    const T *dn = (it & 1) ? dA : dB;   // written by the product of iteration it
    double s[1] = {0.0};
    const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kVecPerThread; ++j) {
        const int64_t i = base + j * kBlock;
        if (i < n) {
            x[i] = fmaT<T>(alpha, dn[i], x[i]);
            const T rv = fmaT<T>(-alpha, q[i], r[i]);
            r[i] = rv;
            s[0] = fma((double)rv, (double)rv, s[0]);
        }
    }
    double out[1];
    if (grid_reduce<1>(s, part, &st->tk_upd, gridDim.x, blockIdx.x, out) && threadIdx.x == 0) {
        const double gnew = out[0], gold = st->gamma;
        if (it < st->k0rec && it < kK0Max) st->ratios[it] = sqrt(gnew) / sqrt(gold);
        st->beta = (double)(T)(gnew / gold);
        st->gamma = gnew;
        st->iter = it + 1;
        if (sqrt(gnew) <= st->thr) {
            st->live = 0; st->reason = kConverged;
        } else if (it + 1 >= st->maxit) {
            st->live = 0; st->reason = kMaxit;
        }
    }
}

template <typename T>
void launch_cg_update(hipStream_t s, int32_t n, T *x, T *r, const T *q, const T *dA, const T *dB,
                      double *part, DevState *st)
{
    const int grid = (n + kVecTile - 1) / kVecTile;
    hipLaunchKernelGGL(k_update<T>, dim3(grid), dim3(kBlock), 0, s, n, x, r, q, dA, dB, part, st);
}

template void launch_cg_spmv<float>(hipStream_t, const int32_t *, const int32_t *, const float *,
                                    int32_t, int, const float *, float *, float *, float *, double *,
                                    DevState *);
template void launch_cg_spmv<double>(hipStream_t, const int32_t *, const int32_t *, const double *,
                                     int32_t, int, const double *, double *, double *, double *,
                                     double *, DevState *);
template void launch_cg_update<float>(hipStream_t, int32_t, float *, float *, const float *,
                                      const float *, const float *, double *, DevState *);
template void launch_cg_update<double>(hipStream_t, int32_t, double *, double *, const double *,
                                       const double *, const double *, double *, DevState *);
template void launch_spmv_plain<float>(hipStream_t, const int32_t *, const int32_t *, const float *,
                                       int32_t, int, const float *, float *);
template void launch_spmv_plain<double>(hipStream_t, const int32_t *, const int32_t *,
                                        const double *, int32_t, int, const double *, double *);

}  // namespace mpcg
