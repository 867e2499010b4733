// The Jacobi method as a second two-stage solver (the section on the matrix
// graph diameter and rounding-error growth in other iterative methods):
// x_{k+1} = D^{-1} (b - (L + U) x_k), A = L + D + U, first in FP32 on the FP32
// copy of A to a relative residual eps1, then in FP64 from float64(x~) to
// eps2 -- Algorithm I with the Jacobi iteration in place of CG.
//
// One launch per iteration.  For every row the off-diagonal sum
// s = sum_{j != i} a_ij x_j is one fma chain in the row's stored order (the
// diagonal entry skipped), t = b_i - s, the residual of the current iterate
// r_i = t - a_ii x_i (one fma) and the next iterate x_{k+1,i} = t / a_ii: the
// residual for the stop test comes from the same gather as the update.
// Launch k reads x_k from xs[k & 1], writes x_{k+1} to xs[(k + 1) & 1] and the
// per-block partials of ||r_k||^2 (FP64) to part[k & 1].  Its prologue
// reduces launch k - 1's partials in a fixed order in every block (no
// cross-block synchronisation): ||r_{k-1}|| <= thr, a non-finite norm or
// k - 1 = maxit ends the stage with x_{k-1}; block 0 records it.  Launch 0
// reduces instead the partials of ||b||^2 (part[1], from k_jac_bnorm) and
// sets the threshold.

#include "mpcg_internal.hpp"
#include "sell_common.hpp"

namespace mpcg {

template <typename T>
struct JacArgs {
    // SELL-64 copy (SELL kernel) or CSR (CSR kernel)
    const int32_t *rp;
    const void *scol;
    const T *sval;
    const int64_t *off;
    const int32_t *col;
    const T *val;
    int32_t n, nslices;
    int32_t k, maxit, abs_tol, np;
    double eps;
    const T *b;
    const T *dg;
    T *x0, *x1;       // xs[0], xs[1]
    double *part;     // 2 * np partials
    DevState *st;
};

// Stop decision of launch k (block-uniform); returns true when the block exits.
template <typename T>
__device__ inline bool jac_prologue(const JacArgs<T> &a, double *sm)
{
    __shared__ int s_skip;
    DevState *st = a.st;
    const int k = a.k;
    if (threadIdx.x == 0) s_skip = st->stop_it < k;
    __syncthreads();
    if (s_skip) return true;
    if (k == 0) {
        const double bb = sell_reduce_partials(a.part + a.np, a.np, sm);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->bnorm2 = bb;
            st->thr = a.abs_tol ? a.eps : a.eps * sqrt(bb);
        }
        return false;
    }
    const double g = sell_reduce_partials(a.part + (size_t)((k - 1) & 1) * a.np, a.np, sm);
    const bool bad = !(g == g) || isinf(g);
    const bool conv = !bad && sqrt(g) <= st->thr;
    const bool cap = !conv && !bad && k - 1 >= a.maxit;
    if (!(conv || cap || bad)) return false;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->gamma = g;
        st->iter = k - 1;
        st->reason = conv ? kConverged : (bad ? kNonFinite : kMaxit);
        st->stop_it = k - 1;
        st->live = 0;
    }
    return true;
}

// NT: nontemporal loads of the matrix stream (see the SELL products)
template <bool NT, typename P> __device__ inline P jac_ld(const P *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <typename T, typename IDX, int B, bool NT>
__global__ void __launch_bounds__(kBlock) k_jac_sell(JacArgs<T> a)
{
    __shared__ double sm[kBlock / 64 + 1];
    if (jac_prologue<T>(a, sm)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const T *x = (a.k & 1) ? a.x1 : a.x0;
    T *xn = (a.k & 1) ? a.x0 : a.x1;
    const IDX *scol = static_cast<const IDX *>(a.scol);
    double s2 = 0.0;
    for (SliceWalk w = slice_walk(a.nslices); w.g < w.g_end; w.g += w.step) {
        const int sl = w.g * (kBlock / 64) + wv;
        if (sl >= a.nslices) continue;
        const int row = sl * 64 + lane;
        const bool has = row < a.n;
        const int len = has ? a.rp[row + 1] - a.rp[row] : 0;
        const int64_t base = a.off[sl];
        const int W = (int)((a.off[sl + 1] - base) >> 6);
        const IDX *cp = scol + base + lane;
        const T *vp = a.sval + base + lane;
        const int safe = has ? row : a.n - 1;
        T acc = T(0);
        for (int k0 = 0; k0 < W; k0 += B) {
            int c[B];
            T v[B], g[B];
            if (sizeof(T) == 4) {
                // FP32: every lane loads the whole batch (an entry past the
                // row's length is the slice's padding, past W its last column,
                // both inside the slice; it gathers the row itself), so the
                // batch's loads and gathers are issued together
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int kk = k0 + j < W ? k0 + j : W - 1;
                    const IDX ci = jac_ld<NT>(cp + (int64_t)kk * 64);
                    v[j] = jac_ld<NT>(vp + (int64_t)kk * 64);
                    const int cc = (sizeof(IDX) == 2) ? row + (int)ci : (int)ci;
                    c[j] = k0 + j < len ? cc : row;
                    g[j] = x[k0 + j < len ? cc : safe];
                }
            } else {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    c[j] = row;
                    if (k0 + j < len) {
                        const IDX ci = jac_ld<NT>(cp + (int64_t)(k0 + j) * 64);
                        c[j] = (sizeof(IDX) == 2) ? row + (int)ci : (int)ci;
                        v[j] = jac_ld<NT>(vp + (int64_t)(k0 + j) * 64);
                    }
                }
#pragma unroll
                for (int j = 0; j < B; ++j)
                    if (k0 + j < len && c[j] != row) g[j] = x[c[j]];
            }
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (k0 + j < len && c[j] != row) acc = fma_t<T>(v[j], g[j], acc);
        }
        if (has) {
            const T d = a.dg[row];
            const T t = a.b[row] - acc;
            const T r = fma_t<T>(-d, x[row], t);
            xn[row] = t / d;
            s2 = fma((double)r, (double)r, s2);
        }
    }
    const double bs = sell_block_sum(s2, sm);
    if (tid == 0) a.part[(size_t)(a.k & 1) * a.np + blockIdx.x] = bs;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_jac_csr(JacArgs<T> a)
{
    __shared__ double sm[kBlock / 64 + 1];
    if (jac_prologue<T>(a, sm)) return;
    const T *x = (a.k & 1) ? a.x1 : a.x0;
    T *xn = (a.k & 1) ? a.x0 : a.x1;
    double s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        T acc = T(0);
        for (int32_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int c = a.col[e];
            if (c != i) acc = fma_t<T>(a.val[e], x[c], acc);
        }
        const T d = a.dg[i];
        const T t = a.b[i] - acc;
        const T r = fma_t<T>(-d, x[i], t);
        xn[i] = t / d;
        s2 = fma((double)r, (double)r, s2);
    }
    const double bs = sell_block_sum(s2, sm);
    if (threadIdx.x == 0) a.part[(size_t)(a.k & 1) * a.np + blockIdx.x] = bs;
}

// partials of ||b||^2 (FP64) into part[np + block], np = gridDim.x
__global__ void __launch_bounds__(kBlock) k_jac_bnorm(const double *b, int32_t n, double *part, int32_t np)
{
    __shared__ double sm[kBlock / 64 + 1];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s = fma(b[i], b[i], s);
    const double bs = sell_block_sum(s, sm);
    if (threadIdx.x == 0) part[np + blockIdx.x] = bs;
}

__global__ void k_jac_start(DevState *st)
{
    if (threadIdx.x == 0) {
        st->stop_it = kNoStop;
        st->live = 1;
        st->iter = 0;
        st->reason = 0;
        st->gamma = 0.0;
    }
}

__global__ void k_jac_widen(const float *x32, double *x64, int32_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x64[i] = (double)x32[i];
}

int jacobi_grid(const JacMat &m)
{
    if (m.use_sell) return m.sell.grid;
    int g = (m.n + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    return g < 1 ? 1 : g;
}

void launch_jacobi_begin(hipStream_t s, const JacMat &m, const double *b, double *part, DevState *st)
{
    const int np = jacobi_grid(m);
    hipLaunchKernelGGL(k_jac_bnorm, dim3(np), dim3(kBlock), 0, s, b, m.n, part, np);
    hipLaunchKernelGGL(k_jac_start, dim3(1), dim3(64), 0, s, st);
}

template <typename T>
void launch_jacobi_iter(hipStream_t s, const JacMat &m, const T *val_csr, const T *b, const T *dg, T *x0, T *x1,
                        int k, int maxit, double eps, int abs_tol, double *part, DevState *st)
{
    JacArgs<T> a{};
    a.rp = m.rp;
    a.n = m.n;
    a.k = k;
    a.maxit = maxit;
    a.abs_tol = abs_tol;
    a.eps = eps;
    a.np = jacobi_grid(m);
    a.b = b;
    a.dg = dg;
    a.x0 = x0;
    a.x1 = x1;
    a.part = part;
    a.st = st;
    if (m.use_sell) {
        a.scol = m.sell.scol;
        a.sval = sizeof(T) == 8 ? reinterpret_cast<const T *>(m.sell.v64) : reinterpret_cast<const T *>(m.sell.v32);
        a.off = m.sell.off;
        a.nslices = m.sell.nslices;
        const bool nt = (m.sell.nt_mask >> (sizeof(T) == 8 ? 1 : 0)) & 1;
        if (m.sell.idx16) {
            if (nt) hipLaunchKernelGGL((k_jac_sell<T, int16_t, 4, true>), dim3(a.np), dim3(kBlock), 0, s, a);
            else hipLaunchKernelGGL((k_jac_sell<T, int16_t, 4, false>), dim3(a.np), dim3(kBlock), 0, s, a);
        } else {
            if (nt) hipLaunchKernelGGL((k_jac_sell<T, int32_t, 4, true>), dim3(a.np), dim3(kBlock), 0, s, a);
            else hipLaunchKernelGGL((k_jac_sell<T, int32_t, 4, false>), dim3(a.np), dim3(kBlock), 0, s, a);
        }
    } else {
        a.col = m.col;
        a.val = val_csr;
        hipLaunchKernelGGL((k_jac_csr<T>), dim3(a.np), dim3(kBlock), 0, s, a);
    }
}

void launch_jacobi_widen(hipStream_t s, const float *x32, double *x64, int32_t n)
{
    int g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_jac_widen, dim3(g), dim3(kBlock), 0, s, x32, x64, n);
}

template void launch_jacobi_iter<float>(hipStream_t, const JacMat &, const float *, const float *, const float *,
                                        float *, float *, int, int, double, int, double *, DevState *);
template void launch_jacobi_iter<double>(hipStream_t, const JacMat &, const double *, const double *,
                                         const double *, double *, double *, int, int, double, int, double *,
                                         DevState *);

}  // namespace mpcg
