// Integer frontier BFS for the 2BFS pseudo-diameter (section "Computing
// Pseudo-Diameter of the Graph Matrix"), per connected component.
//
// Distances are unique, so the result is bit-exact whatever the order in
// which a level is expanded; the farthest vertex is the smallest index among
// the vertices at the largest distance.
//
// A BFS "round" is one launch of the one-workgroup kernel (runs many levels
// back to back while the frontier fits in LDS, which covers long thin graphs
// such as bands) followed by a number of multi-block level launches (used
// while the frontier is large).  Each launch reads the frontier state from
// device memory and exits at once when it is not its turn, so the host can
// enqueue rounds without waiting for every level.

#include "mpcg_internal.hpp"

namespace mpcg {

constexpr int kIntMax = 0x7fffffff;

__device__ inline int atomic_load_i32(const int32_t *p)
{
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ seeding --

__global__ void k_bfs_seed_single(int32_t *dist, int32_t *q0, int32_t src, DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dist[src] = 0;
        q0[0] = src;
        st->bfs_level = 0;
        st->bfs_cur = 1;
        st->bfs_next = 0;
        st->bfs_parity = 0;
        st->bfs_done = 0;
        st->bfs_cur_min = src;
        st->bfs_next_min = kIntMax;
        st->bfs_far = src;
        st->bfs_visited = 1;
        st->tk_bfs = 0;
    }
}

void launch_bfs_seed_single(hipStream_t s, const BfsBufs &b, int32_t src)
{
    launch_fill_i32(s, b.dist, b.n, -1);
    hipLaunchKernelGGL(k_bfs_seed_single, dim3(1), dim3(64), 0, s, b.dist, b.q0, src, b.st);
}

// ------------------------------------------------- one-workgroup rounds --

// Runs levels while 0 < frontier <= small_max (<= kBfsSmallCap, chosen so
// that one pass of the 1024 threads covers the level).  The frontier lives in LDS;
// the next frontier is also written to the global queue so that the
// multi-block kernel can take over when it outgrows LDS.
__global__ void __launch_bounds__(kBfsSmallThreads)
k_bfs_small(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *dist,
            int32_t *q0, int32_t *q1, int32_t n, int32_t lanes, int32_t small_max, DevState *st)
{
    __shared__ int32_t sq[2][kBfsSmallCap];
    __shared__ int32_t s_cnt, s_min, s_cur, s_level, s_par, s_go, s_curmin;
    __shared__ long long s_vis;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const int cur = st->bfs_cur;
        s_go = (!st->bfs_done && cur > 0 && cur <= small_max) ? 1 : 0;
        s_cur = cur;
        s_level = st->bfs_level;
        s_par = st->bfs_parity;
        s_curmin = st->bfs_cur_min;
        s_vis = st->bfs_visited;
    }
    __syncthreads();
    if (!s_go) return;
    {
        const int32_t *qc = s_par ? q1 : q0;
        for (int i = tid; i < s_cur; i += kBfsSmallThreads) sq[0][i] = qc[i];
    }
    int c = 0;
    bool finished = false;
    // every iteration expands one level; at most n levels exist
    for (;;) {
        if (tid == 0) { s_cnt = 0; s_min = kIntMax; }
        __syncthreads();
        const int cur = s_cur, level = s_level;
        int32_t *qn = s_par ? q0 : q1;
        const int work = cur * lanes;
        for (int w = tid; w < work; w += kBfsSmallThreads) {
            const int f = w / lanes, l = w - f * lanes;
            const int u = sq[c][f];
            if ((unsigned)u >= (unsigned)n) continue;
            const int e = rp[u + 1];
            for (int k = rp[u] + l; k < e; k += lanes) {
                const int v = col[k];
                if (v == u || dist[v] >= 0) continue;
                if (atomicCAS(&dist[v], -1, level + 1) == -1) {
                    const int pos = atomicAdd(&s_cnt, 1);
                    if (pos < kBfsSmallCap) sq[c ^ 1][pos] = v;
                    qn[pos] = v;
                    atomicMin(&s_min, v);
                }
            }
        }
        __syncthreads();
        const int nxt = s_cnt;
        if (nxt == 0) { finished = true; break; }
        if (tid == 0) {
            s_vis += nxt;
            s_level = level + 1;
            s_par ^= 1;
            s_cur = nxt;
            s_curmin = s_min;
        }
        c ^= 1;
        __syncthreads();
        if (nxt > small_max) break;
    }
    if (tid == 0) {
        st->bfs_level = s_level;
        st->bfs_cur = finished ? 0 : s_cur;
        st->bfs_parity = s_par;
        st->bfs_cur_min = s_curmin;
        st->bfs_visited = s_vis;
        st->bfs_next = 0;
        st->bfs_next_min = kIntMax;
        if (finished) {
            st->bfs_done = 1;
            st->bfs_far = s_curmin;
        }
    }
}

// ----------------------------------------------------- multi-block level --

__device__ inline int wave_max_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}
__device__ inline int wave_min_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = v < o ? v : o;
    }
    return v;
}

// One level, top-down.  `lanes` consecutive lanes share a frontier vertex
// and take its neighbours in parallel (lane l: entries l, l + lanes, ...);
// every wave runs a wave-uniform loop so that appends to the next frontier
// take one atomic per wave and step.
__global__ void __launch_bounds__(kBlock)
k_bfs_level(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *dist,
            int32_t *q0, int32_t *q1, int32_t n, int32_t lanes, int32_t small_max, DevState *st)
{
    const int cur = min(st->bfs_cur, n);
    if (st->bfs_done || cur <= small_max) return;
    const int level = st->bfs_level;
    const int par = st->bfs_parity;
    const int32_t *qc = par ? q1 : q0;
    int32_t *qn = par ? q0 : q1;
    const int lane = threadIdx.x & 63;
    int wmin = kIntMax;
    const int64_t items = (int64_t)cur * lanes;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t wbase = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); wbase < items; wbase += stride) {
        const int64_t w = wbase + lane;
        int u = -1, k = 0, e = 0;
        if (w < items) {
            const int f = (int)(w / lanes), l = (int)(w - (int64_t)f * lanes);
            u = qc[f];
            if ((unsigned)u < (unsigned)n) {
                k = rp[u] + l;
                e = rp[u + 1];
            }
        }
        int steps = k < e ? (e - k + lanes - 1) / lanes : 0;
        steps = wave_max_i(steps);
        for (int j = 0; j < steps; ++j, k += lanes) {
            int v = -1;
            bool found = false;
            if (k < e) {
                v = col[k];
                if (v != u && dist[v] < 0) found = (atomicCAS(&dist[v], -1, level + 1) == -1);
            }
            const unsigned long long m = __ballot(found);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&st->bfs_next, __popcll(m));
                base = __shfl(base, leader, 64);
                if (found) {
                    const int off = __popcll(m & ((1ull << lane) - 1ull));
                    qn[base + off] = v;
                    wmin = wmin < v ? wmin : v;
                }
            }
        }
    }
    wmin = wave_min_i(wmin);
    // The last block to arrive only needs the two atomic counters, so the
    // arrival ticket needs no memory fence: every block's counter updates are
    // returning atomics, complete before its ticket increment is issued.
    __shared__ int amlast, sink;
    if (lane == 0 && wmin != kIntMax)
        sink = __hip_atomic_fetch_min(&st->bfs_next_min, wmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&st->tk_bfs, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        amlast = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (amlast && threadIdx.x == 0) {
        const int nxt = atomic_load_i32(&st->bfs_next);
        const int nmin = atomic_load_i32(&st->bfs_next_min);
        if (nxt == 0) {
            st->bfs_done = 1;
            st->bfs_cur = 0;
            st->bfs_far = st->bfs_cur_min;
        } else {
            st->bfs_visited += nxt;
            st->bfs_level = level + 1;
            st->bfs_cur = nxt;
            st->bfs_cur_min = nmin;
            st->bfs_parity = par ^ 1;
        }
        st->bfs_next = 0;
        st->bfs_next_min = kIntMax;
        __hip_atomic_store(&st->tk_bfs, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

void launch_bfs_round(hipStream_t s, const BfsBufs &b, int levels)
{
    hipLaunchKernelGGL(k_bfs_small, dim3(1), dim3(kBfsSmallThreads), 0, s, b.rp, b.col, b.dist, b.q0,
                       b.q1, b.n, b.lanes, b.small_max, b.st);
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > kBfsLevelBlocks) grid = kBfsLevelBlocks;
    for (int l = 0; l < levels; ++l)
        hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(kBlock), 0, s, b.rp, b.col, b.dist, b.q0, b.q1,
                           b.n, b.lanes, b.small_max, b.st);
}

// ------------------------------------------------ connected components --

// Lock-free union-find: roots are hooked larger-under-smaller, so the final
// root of every component is its smallest vertex -- the vertex from which a
// sequential scan over s = 0..n-1 would start that component's first sweep.
__device__ inline int cc_find(int32_t *parent, int x)
{
    int p = atomic_load_i32(&parent[x]);
    int guard = 0;
    while (p != x && guard < (1 << 24)) {
        const int pp = atomic_load_i32(&parent[p]);
        if (pp != p) __hip_atomic_store(&parent[x], pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = pp;
        ++guard;
    }
    return x;
}

__global__ void k_cc_init(int32_t *parent, int32_t n)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) parent[i] = i;
}

__global__ void __launch_bounds__(kBlock)
k_cc_hook(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *parent,
          int32_t n, DevState *st)
{
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int e = rp[v + 1];
        for (int k = rp[v]; k < e; ++k) {
            const int u = col[k];
            if (u <= v) continue;   // each undirected edge once
            int tries = 0;
            for (;;) {
                int ru = cc_find(parent, u), rv = cc_find(parent, v);
                if (ru == rv) break;
                if (ru < rv) { const int t = ru; ru = rv; rv = t; }   // hook ru (larger) under rv
                if (atomicCAS(&parent[ru], ru, rv) == ru) break;
                if (++tries > (1 << 20)) { atomicOr(&st->guard, 1); break; }
            }
        }
    }
}

__global__ void k_cc_compress(int32_t *parent, int32_t *label, int32_t n)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        label[i] = cc_find(parent, i);
}

void launch_cc(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    // parent[] lives in tarr; the compressed labels go to label[]
    hipLaunchKernelGGL(k_cc_init, dim3(grid), dim3(kBlock), 0, s, b.tarr, b.n);
    hipLaunchKernelGGL(k_cc_hook, dim3(grid), dim3(kBlock), 0, s, b.rp, b.col, b.tarr, b.n, b.st);
    hipLaunchKernelGGL(k_cc_compress, dim3(grid), dim3(kBlock), 0, s, b.tarr, b.label, b.n);
}

// Multi-source start: every component root (label[v] == v) at distance 0.
__global__ void k_bfs_seed_roots(const int32_t *label, int32_t *dist, int32_t *q0,
                                 unsigned long long *best, int32_t n, DevState *st)
{
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const bool root = label[v] == v;
        dist[v] = root ? 0 : -1;
        if (root) {
            best[v] = 0ull;
            const int pos = atomicAdd(&st->bfs_next, 1);
            q0[pos] = v;
        }
    }
}

__global__ void k_bfs_seed_finish(DevState *st, int roots_in_next)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int cnt = st->bfs_next;
        st->bfs_level = 0;
        st->bfs_cur = cnt;
        st->bfs_next = 0;
        st->bfs_parity = 0;
        st->bfs_done = cnt == 0;
        st->bfs_cur_min = 0;
        st->bfs_next_min = kIntMax;
        st->bfs_visited = cnt;
        st->tk_bfs = 0;
        if (roots_in_next) {
            st->ncomp = cnt;
            st->comp_best = 0ull;
        }
    }
}

__global__ void k_zero_next(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->bfs_next = 0;
}

void launch_bfs_seed_roots(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_zero_next, dim3(1), dim3(64), 0, s, b.st);
    hipLaunchKernelGGL(k_bfs_seed_roots, dim3(grid), dim3(kBlock), 0, s, b.label, b.dist, b.q0, b.best,
                       b.n, b.st);
    hipLaunchKernelGGL(k_bfs_seed_finish, dim3(1), dim3(64), 0, s, b.st, 1);
}

// Per-component farthest vertex: key = (dist << 32) | (0xffffffff - v), so the
// maximum key is the largest distance with the smallest vertex.
__global__ void __launch_bounds__(kBlock)
k_comp_argmax(const int32_t *label, const int32_t *dist, unsigned long long *best, int32_t n)
{
    for (int wbase = blockIdx.x * kBlock + (threadIdx.x & ~63); wbase < n; wbase += gridDim.x * kBlock) {
        const int v = wbase + (threadIdx.x & 63);
        int lab = -1;
        unsigned long long key = 0ull;
        if (v < n && dist[v] >= 0) {
            lab = label[v];
            key = ((unsigned long long)(unsigned)dist[v] << 32) | (unsigned long long)(0xffffffffu - (unsigned)v);
        }
        // fast path: the whole wave belongs to one component
        const int l0 = __shfl(lab, 0, 64);
        const bool same = __all(lab == l0);
        if (same) {
            unsigned long long k = key;
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(k, off, 64);
                k = k > o ? k : o;
            }
            if ((threadIdx.x & 63) == 0 && l0 >= 0) atomicMax(&best[l0], k);
        } else if (lab >= 0) {
            atomicMax(&best[lab], key);
        }
    }
}

void launch_comp_argmax(hipStream_t s, const BfsBufs &b, int second_sweep)
{
    (void)second_sweep;
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_comp_argmax, dim3(grid), dim3(kBlock), 0, s, b.label, b.dist, b.best, b.n);
}

// Second sweep start: t_c of every component (from best[c]) at distance 0;
// tarr[c] keeps t_c, best[c] is reset for the second argmax.
__global__ void k_bfs_seed_far(const int32_t *label, int32_t *dist, int32_t *q0, int32_t *tarr,
                               unsigned long long *best, int32_t n, DevState *st)
{
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        if (label[v] == v) {
            const int t = (int)(0xffffffffu - (unsigned)(best[v] & 0xffffffffull));
            tarr[v] = t;
            best[v] = 0ull;
            dist[t] = 0;
            const int pos = atomicAdd(&st->bfs_next, 1);
            q0[pos] = t;
        }
    }
}

void launch_bfs_seed_far(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    launch_fill_i32(s, b.dist, b.n, -1);
    hipLaunchKernelGGL(k_zero_next, dim3(1), dim3(64), 0, s, b.st);
    hipLaunchKernelGGL(k_bfs_seed_far, dim3(grid), dim3(kBlock), 0, s, b.label, b.dist, b.q0, b.tarr,
                       b.best, b.n, b.st);
    hipLaunchKernelGGL(k_bfs_seed_finish, dim3(1), dim3(64), 0, s, b.st, 0);
}

// Best component: key = (ecc_c << 32) | (0xffffffff - c), maximum = largest
// pseudo-diameter, first component on ties.
__global__ void k_comp_final(const int32_t *label, const unsigned long long *best, int32_t n,
                             DevState *st)
{
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < n; c += gridDim.x * kBlock) {
        if (label[c] == c) {
            const unsigned long long ecc = best[c] >> 32;
            const unsigned long long key = (ecc << 32) | (unsigned long long)(0xffffffffu - (unsigned)c);
            atomicMax(&st->comp_best, key);
        }
    }
}

void launch_comp_final(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_comp_final, dim3(grid), dim3(kBlock), 0, s, b.label, b.best, b.n, b.st);
}

}  // namespace mpcg
