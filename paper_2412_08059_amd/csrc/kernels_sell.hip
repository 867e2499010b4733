// SELL-64 storage and kernels for the CG products (gfx950, wave64).
//
// At ingest the CSR matrix is copied into slices of 64 consecutive rows, one
// row per lane of a wavefront; the k-th entries of the 64 rows are stored
// next to each other (column-major inside the slice), so every load of a
// value or column index is one coalesced 64-wide access.  Each lane still
// walks its own row in CSR order with one fma chain starting from 0 -- the
// same rounding sequence as the sequential row loop -- and the padding past a
// row's length is never touched (per-lane predicate, no dummy fma).
//
// When the matrix bandwidth max|i - j| is below 32768 the column is stored as
// a 16-bit offset from the row (2 bytes instead of 4 per entry).  A CG
// product then moves 10 bytes per entry in FP64 and 6 bytes in FP32.
//
// A wave needs no LDS and no block barrier, so many waves per SIMD hide the
// gather latency.  Blocks walk contiguous, XCD-local ranges of slices.

#include "mpcg_internal.hpp"
#include "sell_common.hpp"

#include <cmath>

namespace mpcg {

// ------------------------------------------------------------- ingest --
//
// Ingest is three launches and one host read-back:
//   k_ingest_rows     thread per row: row-pointer checks (and int64 -> int32
//                     conversion), b finite, row length, bandwidth from the
//                     first and last column of the row, slice width;
//   k_sell_scan       padded slice offsets;
//   k_ingest_entries  wave per slice, entries read in coalesced 64-wide
//                     strides: column range, strictly increasing columns,
//                     finite values, and the SELL-64 copy when it fits.

__global__ void __launch_bounds__(kBlock)
k_ingest_rows(const void *rp_in, int rp_is_i64, const int32_t *__restrict__ col,
              const double *__restrict__ b, int32_t n, int64_t nnz, int32_t nslices,
              int32_t *__restrict__ rp32_out, int64_t *__restrict__ wid, int32_t *__restrict__ blk)
{
    __shared__ int sm[3][kBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int err = 0, len = 0, band = 0;
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
        } else if (hi > lo) {
            len = (int)(hi - lo);
            const int c0 = col[lo], c1 = col[hi - 1];
            if (c0 < 0 || c1 >= n) err |= kErrCol;
            const int64_t d0 = i - (int64_t)c0, d1 = (int64_t)c1 - i;
            int64_t d = d0 > d1 ? d0 : d1;
            if (d < 0) d = -d;
            band = d > 0x3fffffff ? 0x3fffffff : (int)d;
        }
        if (rp32_out) {
            rp32_out[i] = (int32_t)lo;
            if (i == n - 1) rp32_out[n] = (int32_t)hi;
        }
        if (b && !isfinite(b[i])) err |= kErrNonFiniteB;
    }
    for (int off = 32; off > 0; off >>= 1) {
        err |= __shfl_xor(err, off, 64);
        const int ol = __shfl_xor(len, off, 64);
        len = len > ol ? len : ol;
        const int ob = __shfl_xor(band, off, 64);
        band = band > ob ? band : ob;
    }
    // per-block statistics; the scan kernel folds them (no same-address atomics)
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        const int64_t s = i >> 6;
        if (s < nslices) wid[s] = (int64_t)len * 64;
        sm[0][w] = err;
        sm[1][w] = len;
        sm[2][w] = band;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int e = 0, l = 0, bd = 0;
        for (int j = 0; j < kBlock / 64; ++j) {
            e |= sm[0][j];
            l = l > sm[1][j] ? l : sm[1][j];
            bd = bd > sm[2][j] ? bd : sm[2][j];
        }
        blk[3 * blockIdx.x] = e;
        blk[3 * blockIdx.x + 1] = l;
        blk[3 * blockIdx.x + 2] = bd;
    }
}

// exclusive scan of the padded slice sizes (one block), off[nslices] = total;
// also folds the per-block ingest statistics into the device state
__global__ void __launch_bounds__(1024)
k_sell_scan(const int64_t *wid, int32_t nslices, int64_t *off, const int32_t *blk, int32_t nblk,
            DevState *st)
{
    __shared__ int64_t part[1024];
    __shared__ int fold[3][1024];
    const int t = threadIdx.x;
    {
        int e = 0, l = 0, bd = 0;
        for (int i = t; i < nblk; i += 1024) {
            e |= blk[3 * i];
            l = l > blk[3 * i + 1] ? l : blk[3 * i + 1];
            bd = bd > blk[3 * i + 2] ? bd : blk[3 * i + 2];
        }
        fold[0][t] = e;
        fold[1][t] = l;
        fold[2][t] = bd;
        __syncthreads();
        for (int d = 512; d > 0; d >>= 1) {
            if (t < d) {
                fold[0][t] |= fold[0][t + d];
                fold[1][t] = fold[1][t] > fold[1][t + d] ? fold[1][t] : fold[1][t + d];
                fold[2][t] = fold[2][t] > fold[2][t + d] ? fold[2][t] : fold[2][t + d];
            }
            __syncthreads();
        }
        if (t == 0) {
            st->ing_err |= fold[0][0];
            st->max_row = fold[1][0];
            st->max_band = fold[2][0];
        }
    }
    const int per = (nslices + 1023) / 1024;
    const int a = min(t * per, nslices), b = min(a + per, nslices);
    int64_t sum = 0;
    for (int i = a; i < b; ++i) sum += wid[i];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int i = a; i < b; ++i) {
        off[i] = run;
        run += wid[i];
    }
    if (t == 1023) off[nslices] = part[1023];
}

__global__ void __launch_bounds__(kBlock)
k_ingest_entries(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                 const double *__restrict__ val, int32_t n, int32_t nslices,
                 const int64_t *__restrict__ off, int64_t cap, int allow_fill, void *scol,
                 double *__restrict__ sv64, float *__restrict__ sv32, DevState *st)
{
    __shared__ int s_ok;
    if (threadIdx.x == 0) s_ok = !(st->ing_err & kErrRowPtr);
    __syncthreads();
    if (!s_ok) return;   // row pointers are not usable
    const bool fill = allow_fill && off[nslices] <= cap;
    const bool idx16 = st->max_band < 32768;
    const int lane = threadIdx.x & 63;
    int err = 0;
    for (int s = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); s < nslices; s += gridDim.x * (kBlock / 64)) {
        const int r0 = s * 64;
        const int nrows = min(64, n - r0);
        const int rpl = rp[r0 + min(lane, nrows)];      // start of row r0 + lane
        const int lo = __shfl(rpl, 0, 64);
        const int hi = rp[r0 + nrows];
        const int64_t base_off = fill ? off[s] : 0;
        for (int kb = lo; kb < hi; kb += 64) {          // wave-uniform trip count
            const int k = kb + lane;
            // row of entry k: largest m < nrows with rp[r0 + m] <= k
            int m = 0;
            for (int step = 32; step > 0; step >>= 1) {
                const int cand = m + step;
                const int v = __shfl(rpl, cand < 64 ? cand : 63, 64);
                if (cand < nrows && v <= k) m = cand;
            }
            const int rstart = __shfl(rpl, m, 64);
            if (k < hi) {
                const int row = r0 + m;
                const int pos = k - rstart;
                const int c = col[k];
                if (c < 0 || c >= n) err |= kErrCol;
                if (pos > 0 && c <= col[k - 1]) err |= kErrUnsorted;
                const double v = val[k];
                if (!isfinite(v)) err |= kErrNonFiniteA;
                if (fill) {
                    const int64_t dst = base_off + (int64_t)pos * 64 + m;
                    if (idx16) static_cast<int16_t *>(scol)[dst] = (int16_t)(c - row);
                    else static_cast<int32_t *>(scol)[dst] = c;
                    sv64[dst] = v;
                    if (sv32) sv32[dst] = (float)v;
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if (lane == 0 && err) atomicOr(&st->ing_err, err);
}

void launch_ingest_sell(hipStream_t s, const void *rp_in, int rp_is_i64, const int32_t *rp32,
                        int32_t *rp32_out, const int32_t *col, const double *val, const double *b,
                        int32_t n, int64_t nnz, int64_t *wid, int64_t *off, int32_t *blk, int64_t cap,
                        int allow_fill, void *scol, double *sv64, float *sv32, DevState *st)
{
    const int nslices = (n + 63) / 64;
    const int nblk = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_ingest_rows, dim3(nblk), dim3(kBlock), 0, s, rp_in, rp_is_i64, col, b, n, nnz,
                       nslices, rp32_out, wid, blk);
    hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, s, wid, nslices, off, blk, nblk, st);
    int g = (nslices + 3) / 4;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_ingest_entries, dim3(g), dim3(kBlock), 0, s, rp32, col, val, n, nslices, off, cap,
                       allow_fill, scol, sv64, sv32, st);
}

// -------------------------------------------------------------- kernels --

// kSellDir + kSellCgD: the CG product split in two launches for matrices
// whose gathers are scattered (32-bit columns): the first takes the prologue
// of kSellCg and forms d = r + beta d_old (and the deferred x update) row by
// row, the second gathers only d.  The arithmetic is that of kSellCg; a
// scattered gather of one vector instead of two is what it saves.
enum SellMode { kSellCg = 0, kSellRestart = 1, kSellResid = 2, kSellPlain = 3, kSellDir = 4, kSellCgD = 5 };

template <typename T>
struct SellArgs {
    const int32_t *rp;
    const void *scol;
    const T *sval;
    const int64_t *off;
    int32_t n, nslices;
    int32_t it, it0;
    const T *r;
    T *dA, *dB, *q;
    const double *up;
    int32_t nup;
    const float *x32;
    const double *x64in;
    double *x64out;
    const double *b;
    double *rout;
    double *dzA, *dzB;
    const T *xin;
    T *yout;
    T *x;        // CG iterate: receives the deferred alpha_{it-1} d_{it-1}
    T *snap;     // x~ copies at the run-ahead crossings (FP32 only)
    int32_t pc;          // Jacobi: the update partials hold rho (slot b) and r.r (slot nup + b)
    const double *dg;    // restart with Jacobi: diag(A) and z = r / diag(A)
    double *z;
    double *part;
    DevState *st;
};

// NT: the matrix (values, column offsets) is read with nontemporal loads.
// Streamed once per product, it then does not evict the gathered vectors from
// the caches; worth it when the copy exceeds the 256 MB Infinity Cache (a
// copy that fits is re-read from it by the next product).
template <bool NT, typename P> __device__ inline P sell_ld(const P *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// B = entries of a row whose loads are issued together (4 or 8)
// BF: every lane loads all B entries of a batch (no guard per entry), so the
// batch's index and value loads are issued together and its gathers too; an
// entry past the row's length is the slice's padding (past W, its last
// column; both inside the slice), its gather reads the row itself and its
// product is skipped.  Without BF each entry's loads sit behind its own guard.
template <int MODE, typename T, typename IDX, int B, bool BF, bool NT>
__global__ void __launch_bounds__(kBlock) k_sell(SellArgs<T> a)
{
    constexpr int NV = (MODE == kSellRestart) ? 3 : 1;
    __shared__ double sm[kBlock / 64 + 1];
    DevState *st = a.st;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    T beta = T(0), alpha_prev = T(0);
    bool x_pending = false;   // x += alpha_{it-1} d_{it-1} still to apply in the main loop
    const T *dold = nullptr;
    T *dnew = nullptr;
    // dot_acc = 1: the FP32 phase's dot products accumulate in FP32
    const bool f32acc = (MODE == kSellCg || MODE == kSellDir || MODE == kSellCgD) && sizeof(T) == 4 && st->acc32;
    if (MODE == kSellCgD) {   // the direction is formed: skip only after a stop
        __shared__ int s_skip2;
        if (tid == 0) s_skip2 = st->stop_it <= a.it;
        __syncthreads();
        if (s_skip2) return;
        dold = (a.it & 1) ? a.dA : a.dB;   // the d formed by kSellDir of this iteration
    }
    if (MODE == kSellCg || MODE == kSellDir) {
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
            const double rho = f32acc ? sell_reduce_partials_f(a.up, a.nup, sm) : sell_reduce_partials(a.up, a.nup, sm);
            const double g = !a.pc ? rho
                             : f32acc ? sell_reduce_partials_f(a.up + a.nup, a.nup, sm)
                                      : sell_reduce_partials(a.up + a.nup, a.nup, sm);
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
                for (SliceWalk w = slice_walk(a.nslices); w.g < w.g_end; w.g += w.step) {
                    const int i = w.g * kBlock + tid;
                    if (i >= a.n) continue;
                    const T xn = xdone ? a.x[i] : fma_t<T>(alpha_prev, dold[i], a.x[i]);
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
    if (MODE == kSellDir) {   // d = r + beta d_old and the deferred x update, row by row
        for (SliceWalk w = slice_walk(a.nslices); w.g < w.g_end; w.g += w.step) {
            const int i = w.g * kBlock + tid;
            if (i >= a.n) continue;
            const T dof = dold[i];
            if (x_pending) a.x[i] = fma_t<T>(alpha_prev, dof, a.x[i]);
            dnew[i] = fma_t<T>(beta, dof, a.r[i]);
        }
        return;
    }

    const IDX *scol = static_cast<const IDX *>(a.scol);
    const int lb = blockIdx.x;   // partial slot (fixed per block, so sums keep one order)
    double s[NV];
    for (int j = 0; j < NV; ++j) s[j] = 0.0;
    float sf = 0.0f;   // d.q in FP32 (dot_acc = 1)

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
            if (BF) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int kk = k0 + j < W ? k0 + j : W - 1;
                    const IDX ci = sell_ld<NT>(cp + (int64_t)kk * 64);
                    v[j] = sell_ld<NT>(vp + (int64_t)kk * 64);
                    const int cc = (sizeof(IDX) == 2) ? row + (int)ci : (int)ci;
                    c[j] = k0 + j < len ? cc : safe;
                }
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    if (MODE == kSellCg) g[j] = fma_t<T>(beta, dold[c[j]], a.r[c[j]]);
                    else if (MODE == kSellCgD) g[j] = dold[c[j]];
                    else if (MODE == kSellPlain) g[j] = a.xin[c[j]];
                    else g[j] = a.x32 ? (T)a.x32[c[j]] : (T)a.x64in[c[j]];
                }
            } else {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    if (k0 + j < len) {
                        const IDX ci = sell_ld<NT>(cp + (int64_t)(k0 + j) * 64);
                        c[j] = (sizeof(IDX) == 2) ? row + (int)ci : (int)ci;
                        v[j] = sell_ld<NT>(vp + (int64_t)(k0 + j) * 64);
                    }
                }
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    if (k0 + j < len) {
                        if (MODE == kSellCg) g[j] = fma_t<T>(beta, dold[c[j]], a.r[c[j]]);
                        else if (MODE == kSellCgD) g[j] = dold[c[j]];
                        else if (MODE == kSellPlain) g[j] = a.xin[c[j]];
                        else g[j] = a.x32 ? (T)a.x32[c[j]] : (T)a.x64in[c[j]];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (k0 + j < len) acc = fma_t<T>(v[j], g[j], acc);
        }
        if (has) {
            if (MODE == kSellPlain) {
                a.yout[row] = acc;
            } else if (MODE == kSellCgD) {
                const T dn = dold[row];
                a.q[row] = acc;
                if (f32acc) sf = fmaf((float)dn, (float)acc, sf);
                else s[0] = fma((double)dn, (double)acc, s[0]);
            } else if (MODE == kSellCg) {
                const T dof = dold[row];
                if (x_pending) a.x[row] = fma_t<T>(alpha_prev, dof, a.x[row]);
                const T dn = fma_t<T>(beta, dof, a.r[row]);
                dnew[row] = dn;
                a.q[row] = acc;
                if (f32acc) sf = fmaf((float)dn, (float)acc, sf);
                else s[0] = fma((double)dn, (double)acc, s[0]);
            } else {
                const double bv = a.b[row];
                const double res = bv - (double)acc;
                if (MODE == kSellRestart) {
                    if (a.x32) a.x64out[row] = (double)a.x32[row];
                    a.rout[row] = res;
                    double *dz = (a.it0 & 1) ? a.dzB : a.dzA;
                    dz[row] = 0.0;
                    s[1] = fma(bv, bv, s[1]);
                    double zv = res;
                    if (a.dg) {
                        zv = res / a.dg[row];
                        a.z[row] = zv;
                    }
                    s[2] = fma(res, zv, s[2]);
                }
                s[0] = fma(res, res, s[0]);
            }
        }
    }
    if (MODE == kSellPlain) return;
    if (f32acc) {
        const float bs = sell_block_sum_f(sf, sm);
        if (tid == 0) a.part[lb] = (double)bs;
        return;
    }
    for (int j = 0; j < NV; ++j) {
        const double bs = sell_block_sum(s[j], sm);
        if (tid == 0) a.part[(size_t)lb * NV + j] = bs;
    }
}

template <int MODE, typename T, bool BF, bool NT>
static void sell_launch_bf(hipStream_t s, const SellMat &m, const SellArgs<T> &a)
{
    if (m.batch == 8) {
        if (m.idx16)
            hipLaunchKernelGGL((k_sell<MODE, T, int16_t, 8, BF, NT>), dim3(m.grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_sell<MODE, T, int32_t, 8, BF, NT>), dim3(m.grid), dim3(kBlock), 0, s, a);
    } else {
        if (m.idx16)
            hipLaunchKernelGGL((k_sell<MODE, T, int16_t, 4, BF, NT>), dim3(m.grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_sell<MODE, T, int32_t, 4, BF, NT>), dim3(m.grid), dim3(kBlock), 0, s, a);
    }
}

template <int MODE, typename T>
static void sell_launch(hipStream_t s, const SellMat &m, const SellArgs<T> &a)
{
    const int bit = sizeof(T) == 8 ? 1 : 0;
    const bool bf = (m.bf_mask >> bit) & 1, nt = MODE != kSellDir && ((m.nt_mask >> bit) & 1);
    if (bf) {
        if (nt) sell_launch_bf<MODE, T, true, true>(s, m, a);
        else sell_launch_bf<MODE, T, true, false>(s, m, a);
    } else {
        if (nt) sell_launch_bf<MODE, T, false, true>(s, m, a);
        else sell_launch_bf<MODE, T, false, false>(s, m, a);
    }
}

template <typename T>
static SellArgs<T> sell_args(const SellMat &m, const T *sval)
{
    SellArgs<T> a{};
    a.rp = m.rp; a.scol = m.scol; a.sval = sval; a.off = m.off; a.n = m.n; a.nslices = m.nslices;
    return a;
}

template <typename T> static const T *sell_vals(const SellMat &m);
template <> const float *sell_vals<float>(const SellMat &m) { return m.v32; }
template <> const double *sell_vals<double>(const SellMat &m) { return m.v64; }

template <typename T>
void launch_sell_cg_spmv(hipStream_t s, const SellMat &m, const T *r, T *dA, T *dB, T *q,
                         const double *up, int nup, double *part, int it, int it0, T *x, T *snap, int pc,
                         DevState *st)
{
    SellArgs<T> a = sell_args<T>(m, sell_vals<T>(m));
    a.it = it; a.it0 = it0; a.r = r; a.dA = dA; a.dB = dB; a.q = q; a.up = up; a.nup = nup;
    a.x = x; a.snap = snap; a.pc = pc;
    a.part = part; a.st = st;
    if (m.split) {
        sell_launch<kSellDir, T>(s, m, a);
        sell_launch<kSellCgD, T>(s, m, a);
    } else {
        sell_launch<kSellCg, T>(s, m, a);
    }
}

void launch_sell_restart(hipStream_t s, const SellMat &m, const float *x32, double *x64,
                         const double *b, double *r, double *dA, double *dB, int it0, const double *dg,
                         double *z, double *part, DevState *st)
{
    SellArgs<double> a = sell_args<double>(m, m.v64);
    a.dg = dg;
    a.z = z;
    a.it0 = it0; a.x32 = x32; a.x64in = x64; a.x64out = x64; a.b = b; a.rout = r; a.dzA = dA; a.dzB = dB;
    a.part = part; a.st = st;
    sell_launch<kSellRestart, double>(s, m, a);
}

void launch_sell_resid(hipStream_t s, const SellMat &m, const double *x64, const double *b,
                       double *part, DevState *st)
{
    SellArgs<double> a = sell_args<double>(m, m.v64);
    a.x64in = x64; a.b = b; a.part = part; a.st = st;
    sell_launch<kSellResid, double>(s, m, a);
}

template <typename T>
void launch_sell_plain(hipStream_t s, const SellMat &m, const T *x, T *y)
{
    SellArgs<T> a = sell_args<T>(m, sell_vals<T>(m));
    a.xin = x; a.yout = y;
    sell_launch<kSellPlain, T>(s, m, a);
}

template void launch_sell_cg_spmv<float>(hipStream_t, const SellMat &, const float *, float *, float *,
                                         float *, const double *, int, double *, int, int, float *,
                                         float *, int, DevState *);
template void launch_sell_cg_spmv<double>(hipStream_t, const SellMat &, const double *, double *,
                                          double *, double *, const double *, int, double *, int, int,
                                          double *, double *, int, DevState *);
template void launch_sell_plain<float>(hipStream_t, const SellMat &, const float *, float *);
template void launch_sell_plain<double>(hipStream_t, const SellMat &, const double *, double *);

}  // namespace mpcg
