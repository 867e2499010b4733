// CG kernels for gfx950: CSR ingest/cast, CSR-stream SpMV with per-row fma
// chains, fused axpy + dot updates, and a single-pass deterministic grid
// reduction that finalises the CG scalars on the device.
//
// One CG iteration i is two launches:
//   k_cg_spmv    gamma_i = r_i.r_i from the update partials of iteration i-1,
//                stop test, beta_i = gamma_i / gamma_{i-1}, decay ratio for v
//                (eq. 13); d_i = r_i + beta_i d_{i-1} (own rows written,
//                gathered columns recomputed on the fly), q = A d_i, partials
//                of d_i.q.
//   k_cg_update  delta_i from those partials, breakdown test,
//                alpha_i = gamma_i / delta_i (rounded to the working
//                precision), x += alpha d_i, r -= alpha q, partials of r.r.
// Every block of a kernel finishes the previous kernel's reduction itself
// (same partials, same order, same bits), so blocks of one grid never wait
// for each other and no cross-block memory fence is needed; block 0 records
// the scalars in the device state for the host.
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

// Block sum delivered to every thread of the block.
__device__ inline double block_sum_all(double v, double *sm)
{
    double s = block_sum(v, sm);
    if (threadIdx.x == 0) sm[kBlock / 64] = s;
    __syncthreads();
    s = sm[kBlock / 64];
    __syncthreads();
    return s;
}

// Sum of component j of cnt partials (stride doubles apart) written by the
// previous kernel, in a fixed order; every block that calls it gets the same
// bits.  Reductions are finished by their consumer this way, so no kernel
// needs blocks of its own grid to communicate.
__device__ inline double reduce_partials(const double *p, int cnt, int stride, int j, double *sm)
{
    // four loads in flight per thread, added in index order (the same bits
    // as one at a time)
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < cnt; i += 4 * kBlock) {
        const double p0 = p[(size_t)i * stride + j], p1 = p[(size_t)(i + kBlock) * stride + j];
        const double p2 = p[(size_t)(i + 2 * kBlock) * stride + j], p3 = p[(size_t)(i + 3 * kBlock) * stride + j];
        acc += p0;
        acc += p1;
        acc += p2;
        acc += p3;
    }
    for (; i < cnt; i += kBlock) acc += p[(size_t)i * stride + j];
    return block_sum_all(acc, sm);
}

// FP32 accumulation (dot_acc = 1): the same tree in float.  Partials are
// stored widened to double (exact) and narrowed back (exact) when reduced.
__device__ inline float wave_sum_f(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline float block_sum_f(float v, double *sm)
{
    v = wave_sum_f(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = (double)v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kBlock / 64; ++i) s += (float)sm[i];
    }
    __syncthreads();
    return s;
}

__device__ inline double reduce_partials_f(const double *p, int cnt, int stride, int j, double *sm)
{
    float acc = 0.0f;
    for (int i = threadIdx.x; i < cnt; i += kBlock) acc += (float)p[(size_t)i * stride + j];
    float s = block_sum_f(acc, sm);
    if (threadIdx.x == 0) sm[kBlock / 64] = (double)s;
    __syncthreads();
    const double r = sm[kBlock / 64];
    __syncthreads();
    return r;
}

// FP32-phase reduction in the precision dot_acc asks for.
__device__ inline double reduce_partials_acc(bool f32, const double *p, int cnt, int stride, int j, double *sm)
{
    return f32 ? reduce_partials_f(p, cnt, stride, j, sm) : reduce_partials(p, cnt, stride, j, sm);
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

__global__ void k_cast32(const double *__restrict__ val, float *__restrict__ val32, int64_t nnz)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kBlock)
        val32[k] = (float)val[k];
}

void launch_cast32(hipStream_t s, const double *val, float *val32, int64_t nnz)
{
    if (nnz <= 0) return;
    int64_t g = (nnz + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_cast32, dim3((int)g), dim3(kBlock), 0, s, val, val32, nnz);
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

int vec_grid(int64_t n)
{
    int64_t g = (n + kVecTile - 1) / kVecTile;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g < 1) g = 1;
    return (int)g;
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
__device__ inline void start_phase(DevState *st, double gamma, double rho, int32_t iter, double eps, int abs_tol,
                                   int32_t maxit)
{
    st->gamma = gamma;
    st->gam[iter & 1] = rho;
    st->gr[iter & 1] = gamma;
    st->iter = iter;
    st->thr = abs_tol ? eps : eps * sqrt(st->bnorm2);
    st->maxit = maxit;
    if (sqrt(gamma) <= st->thr) {
        st->live = 0; st->reason = kConverged;
    } else if (iter >= maxit) {
        st->live = 0; st->reason = kMaxit;
    } else {
        st->live = 1; st->reason = kRunning;
    }
    st->stop_it = st->live ? kNoStop : iter - 1;   // no product of iteration >= iter runs after a stop
    st->x_it = iter;
}

// A phase resumes after a stop in iteration stop_it: x is complete there.
__device__ inline void resume_phase(DevState *st)
{
    st->x_it = st->stop_it != kNoStop ? st->stop_it : -1;
    st->stop_it = kNoStop;
    st->live = 1;
    st->reason = kRunning;
}

// FP32 phase from x~ = 0: r~ = float32(b), old direction = 0, z = r~ / dg
// (Jacobi); partials of r~.r~, b.b and r~.z (r~.r~ without a preconditioner)
// in FP64 for k_fin_init32.
__global__ void __launch_bounds__(kBlock)
k_init32(const double *__restrict__ b, float *__restrict__ x, float *__restrict__ r,
         float *__restrict__ dA, int32_t n, const float *__restrict__ dg, float *__restrict__ z, double *part,
         int acc32)
{
    __shared__ double sm[kBlock / 64 + 1];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    float f0 = 0.0f, f2 = 0.0f;
    const int64_t nchunk = ((int64_t)n + kVecTile - 1) / kVecTile;
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int64_t i = c * kVecTile + j * kBlock + threadIdx.x;
            if (i < n) {
                const double bv = b[i];
                const float rv = (float)bv;
                r[i] = rv;
                x[i] = 0.0f;
                dA[i] = 0.0f;
                if (acc32) f0 = fmaf(rv, rv, f0);
                else s0 = fma((double)rv, (double)rv, s0);
                s1 = fma(bv, bv, s1);
                if (dg) {
                    const float zv = rv / dg[i];
                    z[i] = zv;
                    if (acc32) f2 = fmaf(rv, zv, f2);
                    else s2 = fma((double)rv, (double)zv, s2);
                }
            }
        }
    }
    s0 = acc32 ? (double)block_sum_f(f0, sm) : block_sum(s0, sm);
    s1 = block_sum(s1, sm);
    s2 = dg ? (acc32 ? (double)block_sum_f(f2, sm) : block_sum(s2, sm)) : s0;
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0;
        part[3 * blockIdx.x + 1] = s1;
        part[3 * blockIdx.x + 2] = s2;
    }
}

__global__ void __launch_bounds__(kBlock)
k_fin_init32(const double *part, int cnt, double eps, int abs_tol, int32_t maxit, int32_t k0rec,
             DevState *st, int acc32)
{
    __shared__ double sm[kBlock / 64 + 1];
    const double g = reduce_partials_acc(acc32, part, cnt, 3, 0, sm);
    const double bb = reduce_partials(part, cnt, 3, 1, sm);
    const double rho = reduce_partials_acc(acc32, part, cnt, 3, 2, sm);
    if (threadIdx.x == 0) {
        st->bnorm2 = bb;
        st->k0rec = k0rec;
        st->acc32 = acc32;
        start_phase(st, g, rho, 0, eps, abs_tol, maxit);
    }
}

void launch_init32(hipStream_t s, const double *b, float *x, float *r, float *dA, int32_t n,
                   double eps, int abs_tol, int32_t maxit, int32_t k0rec, const float *dg, float *z,
                   double *part, DevState *st, int acc32)
{
    const int grid = vec_grid(n);
    hipLaunchKernelGGL(k_init32, dim3(grid), dim3(kBlock), 0, s, b, x, r, dA, n, dg, z, part, acc32);
    hipLaunchKernelGGL(k_fin_init32, dim3(1), dim3(kBlock), 0, s, part, grid, eps, abs_tol, maxit, k0rec,
                       st, acc32);
}

// Continue a phase with a new stop test (Algorithm II after the k0 prefix);
// the next product re-derives gamma and applies the test.
__global__ void k_set_phase(DevState *st, double thr, int32_t maxit, int32_t k0rec)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->thr = thr;
        st->maxit = maxit;
        st->k0rec = k0rec;
        st->spec_on = 0;
        resume_phase(st);
    }
}

void launch_set_phase(hipStream_t s, DevState *st, double thr, int32_t maxit, int32_t k0rec)
{
    hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, st, thr, maxit, k0rec);
}

__global__ void k_set_spec(DevState *st, double scale, int32_t k0, int32_t maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double eps[kNumEps] = {1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7};
        for (int t = 0; t < kNumEps; ++t) {
            st->spec_thr[t] = eps[t] * scale;
            st->cross_iter[t] = -1;
            st->cross_gamma[t] = 0.0;
        }
        st->spec_k0 = k0;
        st->spec_on = 1;
        st->thr = st->spec_thr[kNumEps - 1];   // no candidate is tighter: stop there at the latest
        st->maxit = maxit;
        resume_phase(st);
    }
}

void launch_set_spec(hipStream_t s, DevState *st, double scale, int32_t k0, int32_t maxit)
{
    hipLaunchKernelGGL(k_set_spec, dim3(1), dim3(64), 0, s, st, scale, k0, maxit);
}

// Measurement set-up: a live recurrence that no test can stop, finite partials.
__global__ void k_timing_state(DevState *st, double *part, int cnt)
{
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) part[i] = 1e-3;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->gamma = 1.0;
        st->gam[0] = 1.0;
        st->gam[1] = 1.0;
        st->gr[0] = 1.0;
        st->gr[1] = 1.0;
        st->thr = 0.0;
        st->iter = 0;
        st->maxit = 0x7fffffff;
        st->k0rec = 0;
        st->alph[0] = 0.0;
        st->alph[1] = 0.0;
        st->live = 1;
        st->stop_it = kNoStop;
        st->x_it = -1;
        st->reason = kRunning;
    }
}

void launch_timing_state(hipStream_t s, DevState *st, double *part, int cnt)
{
    hipLaunchKernelGGL(k_timing_state, dim3(1), dim3(kBlock), 0, s, st, part, cnt);
}

// ------------------------------------------------------------- CSR-stream --

enum SpmvMode { kModeCg = 0, kModeRestart = 1, kModeResid = 2, kModePlain = 3 };

template <typename T>
struct SpmvArgs {
    const int32_t *rp;
    const int32_t *col;
    const T *val;
    int32_t n;
    int32_t R;         // rows per tile
    int32_t ntiles;
    int32_t it, it0;   // CG iteration and the first iteration of the phase
    int32_t pc;        // Jacobi: the update partials hold rho (slot b) and r.r (slot nup + b)
    const double *dg;  // restart with Jacobi: diag(A) and z = r / diag(A)
    double *z;
    // CG
    const T *r;
    T *dA, *dB, *q;
    const double *up;  // update partials of iteration it-1
    int32_t nup;
    // restart / residual (T = double)
    const float *x32;
    const double *x64in;
    double *x64out;
    const double *b;
    double *rout;
    double *dzA, *dzB;
    // plain
    const T *xin;
    T *yout;
    T *x;              // CG iterate: receives the deferred alpha_{it-1} d_{it-1}
    T *snap;           // x~ copies at the run-ahead crossings (FP32 only)
    double *part;      // this kernel's partials
    DevState *st;
};

// A tile is R consecutive rows; a block walks a contiguous range of tiles.
// Phase 1 streams the tile's entries [rp[row0], rp[row1]) in LDS-sized chunks
// with coalesced col/val loads and gathers the vector entry of each column;
// phase 2 lets thread t run the fma chain of row row0 + t over its entries in
// CSR order, starting from 0 -- the rounding sequence of a sequential row loop.
template <int MODE, typename T>
__global__ void __launch_bounds__(kBlock) k_spmv(SpmvArgs<T> a)
{
    constexpr int CHUNK = kLdsBytes / (2 * (int)sizeof(T));
    constexpr int NV = (MODE == kModeRestart) ? 3 : 1;
    __shared__ T s_val[CHUNK];
    __shared__ T s_x[CHUNK];
    __shared__ double sm[kBlock / 64 + 1];
    DevState *st = a.st;
    const int tid = threadIdx.x;

    T beta = T(0), alpha_prev = T(0);
    bool x_pending = false;   // x += alpha_{it-1} d_{it-1} still to apply in the main loop
    const T *dold = nullptr;
    T *dnew = nullptr;
    const bool f32acc = MODE == kModeCg && sizeof(T) == 4 && st->acc32;   // dot_acc = 1
    if (MODE == kModeCg) {
        const int it = a.it;
        __shared__ int s_skip, s_xdone;
        if (tid == 0) {
            s_skip = st->stop_it < it;
            s_xdone = st->x_it == it;
        }
        __syncthreads();
        if (s_skip) return;
        dold = (it & 1) ? a.dB : a.dA;
        dnew = (it & 1) ? a.dA : a.dB;
        if (it != a.it0) {
            const bool xdone = s_xdone;
            // rho_it (alpha, beta) and gamma_it = r.r (stop test, v); equal without a preconditioner
            const double rho = reduce_partials_acc(f32acc, a.up, a.nup, 1, 0, sm);
            const double g = a.pc ? reduce_partials_acc(f32acc, a.up + a.nup, a.nup, 1, 0, sm) : rho;
            const double gp = st->gr[(it - 1) & 1];
            const double rhop = st->gam[(it - 1) & 1];
            alpha_prev = (T)st->alph[(it - 1) & 1];
            const bool conv = sqrt(g) <= st->thr;
            const bool cap = !conv && it >= st->maxit;
            if (blockIdx.x == 0 && tid == 0) {
                st->gam[it & 1] = rho;
                st->gr[it & 1] = g;
                const int k = it - 1;
                if (k < st->k0rec && k < kK0Max) st->ratios[k] = sqrt(g) / sqrt(gp);
                if (conv || cap) {
                    st->gamma = g;
                    st->iter = it;
                    st->reason = conv ? kConverged : kMaxit;
                    st->stop_it = it;
                    st->live = 0;
                }
            }
            const unsigned cross = a.snap ? spec_crossings(st, it, g) : 0u;
            if (conv || cap || cross) {
                // the iterate x_it of this block's rows, then its run-ahead copies
                const int lb0 = xcd_remap(blockIdx.x, gridDim.x);
                const int r0 = (int)((int64_t)lb0 * a.ntiles / gridDim.x) * a.R;
                const int r1 = min((int)((int64_t)(lb0 + 1) * a.ntiles / gridDim.x) * a.R, a.n);
                for (int i = r0 + tid; i < r1; i += kBlock) {
                    const T xn = xdone ? a.x[i] : fmaT<T>(alpha_prev, dold[i], a.x[i]);
                    if (!xdone) a.x[i] = xn;
                    for (int t = 0; t < kNumEps; ++t)
                        if (cross & (1u << t)) a.snap[(size_t)t * a.n + i] = xn;
                }
                if (blockIdx.x == 0 && tid == 0) {
                    for (int t = 0; t < kNumEps; ++t) {
                        if (!(cross & (1u << t))) continue;
                        st->cross_iter[t] = it;
                        st->cross_gamma[t] = g;
                    }
                }
                if (conv || cap) return;
            } else {
                x_pending = !xdone;
            }
            beta = (T)(rho / rhop);
        }
    }

    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t0 = (int)((int64_t)lb * a.ntiles / gridDim.x);
    const int t1 = (int)((int64_t)(lb + 1) * a.ntiles / gridDim.x);
    double s[NV];
    for (int j = 0; j < NV; ++j) s[j] = 0.0;
    float sf = 0.0f;   // d.q in FP32 (dot_acc = 1)

    for (int t = t0; t < t1; ++t) {
        const int row0 = t * a.R;
        const int row1 = min(row0 + a.R, a.n);
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
        if (has) {
            if (MODE == kModePlain) {
                a.yout[my_row] = acc;
            } else if (MODE == kModeCg) {
                const T dof = dold[my_row];
                if (x_pending) a.x[my_row] = fmaT<T>(alpha_prev, dof, a.x[my_row]);
                const T dn = fmaT<T>(beta, dof, a.r[my_row]);
                dnew[my_row] = dn;
                a.q[my_row] = acc;
                if (f32acc) sf = fmaf((float)dn, (float)acc, sf);
                else s[0] = fma((double)dn, (double)acc, s[0]);
            } else {
                const double bv = a.b[my_row];
                const double res = bv - (double)acc;
                if (MODE == kModeRestart) {
                    if (a.x32) a.x64out[my_row] = (double)a.x32[my_row];
                    a.rout[my_row] = res;
                    double *dz = (a.it0 & 1) ? a.dzB : a.dzA;
                    dz[my_row] = 0.0;
                    s[1] = fma(bv, bv, s[1]);
                    double zv = res;
                    if (a.dg) {
                        zv = res / a.dg[my_row];
                        a.z[my_row] = zv;
                    }
                    s[2] = fma(res, zv, s[2]);
                }
                s[0] = fma(res, res, s[0]);
            }
        }
    }
    if (MODE == kModePlain) return;
    if (f32acc) {
        const float bs = block_sum_f(sf, sm);
        if (tid == 0) a.part[lb] = (double)bs;
        return;
    }
    for (int j = 0; j < NV; ++j) {
        const double bs = block_sum(s[j], sm);
        if (tid == 0) a.part[(size_t)lb * NV + j] = bs;
    }
}

// Finish the restart: ||b||^2, gamma of the fresh residual, stop test.
__global__ void __launch_bounds__(kBlock)
k_fin_restart(const double *part, int cnt, int32_t it0, double eps, int abs_tol, int32_t maxit,
              DevState *st)
{
    __shared__ double sm[kBlock / 64 + 1];
    const double g = reduce_partials(part, cnt, 3, 0, sm);
    const double bb = reduce_partials(part, cnt, 3, 1, sm);
    const double rho = reduce_partials(part, cnt, 3, 2, sm);
    if (threadIdx.x == 0) {
        st->bnorm2 = bb;
        st->k0rec = 0;
        start_phase(st, g, rho, it0, eps, abs_tol, maxit);
    }
}

__global__ void __launch_bounds__(kBlock) k_fin_resid(const double *part, int cnt, DevState *st)
{
    __shared__ double sm[kBlock / 64 + 1];
    const double r2 = reduce_partials(part, cnt, 1, 0, sm);
    if (threadIdx.x == 0) st->resid2 = r2;
}

template <typename T>
static SpmvArgs<T> spmv_args(const SpmvShape &sh, const int32_t *rp, const int32_t *col, const T *val)
{
    SpmvArgs<T> a{};
    a.rp = rp; a.col = col; a.val = val; a.n = sh.n; a.R = sh.R; a.ntiles = sh.ntiles;
    return a;
}

template <typename T>
void launch_cg_spmv(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                    const T *val, const T *r, T *dA, T *dB, T *q, const double *up, int nup,
                    double *part, int it, int it0, T *x, T *snap, int pc, DevState *st)
{
    SpmvArgs<T> a = spmv_args<T>(sh, rp, col, val);
    a.it = it; a.it0 = it0; a.x = x; a.snap = snap; a.pc = pc;
    a.r = r; a.dA = dA; a.dB = dB; a.q = q; a.up = up; a.nup = nup; a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeCg, T>), dim3(sh.grid), dim3(kBlock), 0, s, a);
}

void launch_restart(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                    const double *val, const float *x32, double *x64, const double *b, double *r,
                    double *dA, double *dB, int it0, double eps, int abs_tol, int32_t maxit,
                    const double *dg, double *z, double *part, DevState *st)
{
    SpmvArgs<double> a = spmv_args<double>(sh, rp, col, val);
    a.it0 = it0;
    a.dg = dg;
    a.z = z;
    a.x32 = x32; a.x64in = x64; a.x64out = x64; a.b = b; a.rout = r; a.dzA = dA; a.dzB = dB;
    a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeRestart, double>), dim3(sh.grid), dim3(kBlock), 0, s, a);
    launch_fin_restart(s, part, sh.grid, it0, eps, abs_tol, maxit, st);
}

void launch_fin_restart(hipStream_t s, const double *part, int cnt, int it0, double eps, int abs_tol,
                        int32_t maxit, DevState *st)
{
    hipLaunchKernelGGL(k_fin_restart, dim3(1), dim3(kBlock), 0, s, part, cnt, it0, eps, abs_tol, maxit, st);
}

void launch_fin_resid(hipStream_t s, const double *part, int cnt, DevState *st)
{
    hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kBlock), 0, s, part, cnt, st);
}

void launch_resid(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                  const double *val, const double *x64, const double *b, double *part, DevState *st)
{
    SpmvArgs<double> a = spmv_args<double>(sh, rp, col, val);
    a.x32 = nullptr; a.x64in = x64; a.b = b; a.part = part; a.st = st;
    hipLaunchKernelGGL((k_spmv<kModeResid, double>), dim3(sh.grid), dim3(kBlock), 0, s, a);
    launch_fin_resid(s, part, sh.grid, st);
}

template <typename T>
void launch_spmv_plain(hipStream_t s, const SpmvShape &sh, const int32_t *rp, const int32_t *col,
                       const T *val, const T *x, T *y)
{
    SpmvArgs<T> a = spmv_args<T>(sh, rp, col, val);
    a.xin = x; a.yout = y;
    hipLaunchKernelGGL((k_spmv<kModePlain, T>), dim3(sh.grid), dim3(kBlock), 0, s, a);
}

// ------------------------------------------------------------- update --

// Update of iteration it: alpha = rho_it / delta, r -= alpha q, partials of
// r.r -- or, with Jacobi (PC), z = r / diag(A) and partials of r.z (slot b)
// and r.r (slot nup + b).  x += alpha d is left to the next product, which
// reads d anyway.
// The block's first kUpdPre chunks of r and q (and of diag(A)) depend
// neither on the stop test nor on delta, so they are loaded before both: the
// latencies of the stop flag, of the product's partials and of the vectors
// overlap instead of following each other.  Elements are processed in the
// same order as without the prefetch.
constexpr int kUpdPre = 2;

template <typename T, bool PC>
__global__ void __launch_bounds__(kBlock)
k_cg_update(int32_t n, T *__restrict__ r, const T *__restrict__ q, const double *sp, int nsp, double *up,
            int it, const T *__restrict__ dg, T *__restrict__ z, DevState *st)
{
    __shared__ double sm[kBlock / 64 + 1];
    __shared__ int s_skip;
    const int64_t nchunk = ((int64_t)n + kVecTile - 1) / kVecTile;
    T rv[kUpdPre][kVecPerThread], qv[kUpdPre][kVecPerThread], dv[kUpdPre][kVecPerThread];
#pragma unroll
    for (int p = 0; p < kUpdPre; ++p) {
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int64_t i = ((int64_t)blockIdx.x + (int64_t)p * gridDim.x) * kVecTile + j * kBlock + threadIdx.x;
            rv[p][j] = T(0);
            qv[p][j] = T(0);
            dv[p][j] = T(1);
            if (i < n) {
                rv[p][j] = r[i];
                qv[p][j] = q[i];
                if (PC) dv[p][j] = dg[i];
            }
        }
    }
    if (threadIdx.x == 0) s_skip = st->stop_it <= it;
    const double g = st->gam[it & 1];
    const bool f32acc = sizeof(T) == 4 && st->acc32;   // dot_acc = 1
    // delta: the product's partials in a fixed order (the same bits in every
    // block).  nsp <= kMaxGrid, so every thread's share is issued at once;
    // a share past nsp adds +0.0, which leaves the sum's bits unchanged (the
    // running sum starts at +0.0 and so is never -0.0).
    double acc = 0.0;
    float accf = 0.0f;
    if (f32acc) {
        for (int i = threadIdx.x; i < nsp; i += kBlock) accf += (float)sp[i];
    } else {
        double pv[kMaxGrid / kBlock];
#pragma unroll
        for (int k = 0; k < kMaxGrid / kBlock; ++k) {
            const int i = threadIdx.x + k * kBlock;
            pv[k] = i < nsp ? sp[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kMaxGrid / kBlock; ++k) acc += pv[k];
    }
    __syncthreads();
    if (s_skip) return;
    double delta;
    if (f32acc) {
        const float df = block_sum_f(accf, sm);
        if (threadIdx.x == 0) sm[kBlock / 64] = (double)df;
        __syncthreads();
        delta = sm[kBlock / 64];
        __syncthreads();
    } else {
        // butterfly in each wave, then waves 0..3 in order by every thread:
        // block_sum's bits with one barrier (sm_d is written once)
        __shared__ double sm_d[kBlock / 64];
        const double v = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) sm_d[threadIdx.x >> 6] = v;
        __syncthreads();
        delta = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) delta += sm_d[w];
    }
    if (!isfinite(delta) || !(delta > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->delta = delta;
            st->gamma = st->gr[it & 1];
            st->iter = it;
            st->reason = isfinite(delta) ? kNotSpd : kNonFinite;
            st->stop_it = it;
            st->live = 0;
        }
        return;
    }
    const T alpha = (T)(g / delta);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->delta = delta;
        st->alpha = (double)alpha;
        st->alph[it & 1] = (double)alpha;
    }
    double s = 0.0, s2 = 0.0;
    float sf = 0.0f, s2f = 0.0f;
    auto elem = [&](int64_t i, T r0, T q0, T d0) {
        const T rn = fmaT<T>(-alpha, q0, r0);
        r[i] = rn;
        if (f32acc) s2f = fmaf((float)rn, (float)rn, s2f);
        else s2 = fma((double)rn, (double)rn, s2);
        if (PC) {
            const T zv = rn / d0;
            z[i] = zv;
            if (f32acc) sf = fmaf((float)rn, (float)zv, sf);
            else s = fma((double)rn, (double)zv, s);
        }
    };
#pragma unroll
    for (int p = 0; p < kUpdPre; ++p) {
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int64_t i = ((int64_t)blockIdx.x + (int64_t)p * gridDim.x) * kVecTile + j * kBlock + threadIdx.x;
            if (i < n) elem(i, rv[p][j], qv[p][j], dv[p][j]);
        }
    }
    for (int64_t c = blockIdx.x + (int64_t)kUpdPre * gridDim.x; c < nchunk; c += gridDim.x) {
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int64_t i = c * kVecTile + j * kBlock + threadIdx.x;
            if (i < n) elem(i, r[i], q[i], PC ? dg[i] : T(1));
        }
    }
    if (PC) {
        s = f32acc ? (double)block_sum_f(sf, sm) : block_sum(s, sm);
        s2 = f32acc ? (double)block_sum_f(s2f, sm) : block_sum(s2, sm);
        if (threadIdx.x == 0) {
            up[blockIdx.x] = s;
            up[gridDim.x + blockIdx.x] = s2;
        }
    } else {
        s2 = f32acc ? (double)block_sum_f(s2f, sm) : block_sum(s2, sm);
        if (threadIdx.x == 0) up[blockIdx.x] = s2;
    }
}

template <typename T>
void launch_cg_update(hipStream_t s, int32_t n, T *r, const T *q, const double *sp, int nsp, double *up,
                      int nup, int it, const T *dg, T *z, DevState *st)
{
    if (dg)
        hipLaunchKernelGGL((k_cg_update<T, true>), dim3(nup), dim3(kBlock), 0, s, n, r, q, sp, nsp, up, it, dg, z,
                           st);
    else
        hipLaunchKernelGGL((k_cg_update<T, false>), dim3(nup), dim3(kBlock), 0, s, n, r, q, sp, nsp, up, it, dg,
                           z, st);
}

// Thread per row: the diagonal entry of A (CSR order, columns sorted).
__global__ void __launch_bounds__(kBlock)
k_diag(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const double *__restrict__ val,
       int32_t n, double *dg64, float *dg32, DevState *st)
{
    int bad = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double d = 0.0;
        const int e = rp[i + 1];
        for (int k = rp[i]; k < e; ++k)
            if (col[k] == i) d = val[k];
        dg64[i] = d;
        dg32[i] = (float)d;
        if (!(d > 0.0) || !isfinite(d) || !((float)d > 0.0f) || !isfinite((float)d)) bad = 1;
    }
    if (bad) atomicOr(&st->ing_err, kErrDiag);
}

void launch_diag(hipStream_t s, const int32_t *rp, const int32_t *col, const double *val, int32_t n,
                 double *dg64, float *dg32, DevState *st)
{
    hipLaunchKernelGGL(k_diag, dim3(fill_grid(n)), dim3(kBlock), 0, s, rp, col, val, n, dg64, dg32, st);
}

template void launch_cg_spmv<float>(hipStream_t, const SpmvShape &, const int32_t *, const int32_t *,
                                    const float *, const float *, float *, float *, float *,
                                    const double *, int, double *, int, int, float *, float *, int,
                                    DevState *);
template void launch_cg_spmv<double>(hipStream_t, const SpmvShape &, const int32_t *, const int32_t *,
                                     const double *, const double *, double *, double *, double *,
                                     const double *, int, double *, int, int, double *, double *, int,
                                     DevState *);
template void launch_cg_update<float>(hipStream_t, int32_t, float *, const float *, const double *, int,
                                      double *, int, int, const float *, float *, DevState *);
template void launch_cg_update<double>(hipStream_t, int32_t, double *, const double *, const double *,
                                       int, double *, int, int, const double *, double *, DevState *);
template void launch_spmv_plain<float>(hipStream_t, const SpmvShape &, const int32_t *, const int32_t *,
                                       const float *, const float *, float *);
template void launch_spmv_plain<double>(hipStream_t, const SpmvShape &, const int32_t *,
                                        const int32_t *, const double *, const double *, double *);

}  // namespace mpcg
