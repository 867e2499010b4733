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

// Level 0 holds `cnt0` sources (already in queue 0 with distance 0).
__device__ inline void bfs_start(DevState *st, int cnt0, int min0)
{
    st->bfs_lv[0] = 0;
    st->bfs_lv[1] = 0;
    st->bfs_cnt[0] = cnt0;
    st->bfs_min[0] = min0;
    for (int j = 1; j < 4; ++j) {
        st->bfs_cnt[j] = 0;
        st->bfs_min[j] = kIntMax;
    }
    st->bfs_done = cnt0 == 0;
    st->bfs_ecc = 0;
    st->bfs_far = min0;
    st->bfs_visited = 0;
}

__global__ void k_bfs_seed_single(const int32_t *rp, int32_t *dist, QEnt *q0, int32_t src, DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dist[src] = 0;
        q0[0] = QEnt{rp[src], rp[src + 1]};
        bfs_start(st, 1, src);
    }
}

void launch_bfs_seed_single(hipStream_t s, const BfsBufs &b, int32_t src)
{
    launch_fill_i32(s, b.dist, b.n, -1);
    hipLaunchKernelGGL(k_bfs_seed_single, dim3(1), dim3(64), 0, s, b.rp, b.dist, b.q0, src, b.st);
}

// Level L was expanded by the previous launch and found nothing: the BFS is
// done, with the last non-empty level L - 1.
__device__ inline void bfs_finish(DevState *st, int L)
{
    st->bfs_done = 1;
    st->bfs_ecc = L - 1;
    st->bfs_far = st->bfs_min[(L - 1) & 3];
}

// ------------------------------------------------- one-workgroup rounds --

// Runs levels while 0 < frontier <= small_max (<= kBfsSmallCap, chosen so
// that one pass of the 1024 threads covers the level).  The frontier lives in
// LDS (entries beyond its size go to the global queue); when it outgrows
// small_max the LDS part is written to the global queue and the multi-block
// kernel takes over.  A launch that does not run hands its level on unchanged.
//
// Window cache.  On a long thin graph in its natural ordering (a band, a
// path) the frontier and its neighbours stay inside a narrow range of
// indices, and a level is a handful of vertices: its cost is the chain of
// dependent global loads (columns, distance claim, row pointers).  The kernel
// therefore keeps a window of consecutive rows in LDS -- their row pointers,
// column indices and distances -- and claims and expands vertices inside it
// without touching global memory.  The window is only a cache: a vertex
// outside it takes the global path, and its distances are written back
// (agent-scope atomic stores, read back with agent-scope atomic loads) before
// it moves and before the launch ends.  It moves when the next frontier,
// widened by the largest |i - j| of the matrix, is no longer inside it and
// that widened range is at most a quarter of the window; it is placed ahead
// of the frontier in the direction the frontier moves.
constexpr int kWinRows = 2048;
constexpr int kWinEntries = 16384;

__device__ inline void astore_i32(int32_t *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// Where the window goes for a frontier with vertices in [fmin, fmax]
// (pmax: the previous frontier's largest vertex, -1 if unknown).  mode 0:
// stays; 1: rows [base, base + rows) are read and the window is their longest
// prefix whose entries fit; 2: the same with the longest suffix (the frontier
// moves down).
struct WinPlan {
    int mode, base, rows;
};
__device__ inline WinPlan plan_window(int fmin, int fmax, int pmax, int band, int n, int w0, int nw)
{
    WinPlan p{0, 0, 0};
    const long long lo = (long long)fmin - band, hi = (long long)fmax + band;
    if (nw > 0 && lo >= w0 && hi < (long long)w0 + nw) return p;   // covered
    if ((hi - lo + 1) * 4 > kWinRows) return p;                      // too wide to be worth it
    const long long l0 = lo < 0 ? 0 : lo, h1 = hi >= n ? (long long)n : hi + 1;
    if (pmax >= 0 && fmax < pmax) {
        const long long b0 = h1 - kWinRows < 0 ? 0 : h1 - kWinRows;
        p = WinPlan{2, (int)b0, (int)(h1 - b0)};
    } else {
        const long long b0 = l0 > (long long)n - 1 ? (long long)n - 1 : l0;
        const long long r = (long long)n - b0 < kWinRows ? (long long)n - b0 : kWinRows;
        p = WinPlan{1, (int)b0, (int)r};
    }
    return p;
}

// Bit-parallel levels.  When the matrix's largest |i - j| (band) is at most
// kBitBand and the frontier with that margin lies inside the window, the
// first wave runs levels alone on bitsets of the window's rows, one 32-bit
// word per lane: the next frontier is the union over the offsets d of the
// frontier shifted by +-d and masked by the rows that have an entry at -+d
// (the pattern is symmetric, so a row's entries also say who reaches it),
// minus the visited set.  A level is two lane shuffles and, per offset, two
// funnel shifts (alignbit) and two and-or operations, with no barrier and
// no per-vertex atomics.  Each level's new words go to an LDS ring; when it
// is full, and when the wave stops, the whole block turns the ring into
// distances (a thread per newly visited row finds the slot holding its bit)
// and the wave goes on.  The wave stops when the BFS ends or a new frontier
// vertex comes within band rows of a window edge (the window then moves);
// the block then rebuilds its queue from the frontier bits.
constexpr int kBitBand = 8;
constexpr int kBitWords = kWinRows / 32;   // one word per lane
static_assert(kBitWords == 64, "one 32-bit word of window rows per lane of a wave");
constexpr int kBitRing = 128;
constexpr int kBitDone = 0, kBitMove = 1, kBitFlush = 2;

__device__ inline int wave_sum_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(kBfsSmallThreads)
k_bfs_small(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *dist,
            QEnt *q0, QEnt *q1, int32_t n, int32_t lanes, int32_t small_max, int32_t band, int32_t k,
            DevState *st)
{
    __shared__ QEnt sq[2][kBfsSmallCap];
    __shared__ int32_t w_rp[kWinRows + 1], w_dist[kWinRows], w_col[kWinEntries];
    // next-frontier size, smallest and largest vertex, one slot per level
    // modulo 3: a slot is cleared two levels before it is used again, after
    // a barrier that every thread passed once it had read the slot
    __shared__ int32_t s_cnt[3], s_min[3], s_max[3];
    __shared__ int32_t s_cur, s_level, s_go, s_curmin, s_fit;
    __shared__ long long s_vis;
    // bit-parallel levels: per-offset row masks (bit i of word w: row 32w + i
    // has an entry at -d (b_mp) / +d (b_mm)), frontier and visited words, ring
    __shared__ uint32_t b_mp[kBitBand + 1][kBitWords], b_mm[kBitBand + 1][kBitWords];
    __shared__ uint32_t b_f[kBitWords], b_v[kBitWords], b_vs[kBitWords], b_ring[kBitRing][kBitWords];
    __shared__ int32_t b_code, b_level, b_fmin, b_fmax, b_pmax, b_cnt, b_app, b_used, b_base;
    __shared__ long long b_vis;
    const int tid = threadIdx.x;
    const int lsh = __ffs(lanes) - 1;   // lanes is a power of two
    if (tid == 0) {
        s_go = 0;
        for (int i = 0; i < 3; ++i) {
            s_cnt[i] = 0;
            s_min[i] = kIntMax;
            s_max[i] = -1;
        }
        st->bfs_bar = 0u;   // the persistent kernel of this round starts its barrier count at 0
        if (!st->bfs_done) {
            const int L = st->bfs_lv[k & 1];
            const int cur = st->bfs_cnt[L & 3];
            if (cur == 0) {
                bfs_finish(st, L);
            } else if (cur > small_max) {
                st->bfs_lv[(k + 1) & 1] = L;
            } else {
                s_go = 1;
                s_cur = cur;
                s_level = L;
                s_curmin = st->bfs_min[L & 3];
                s_vis = st->bfs_visited;
            }
        }
    }
    __syncthreads();
    if (!s_go) return;
    // the level state is block-uniform and kept in registers by every thread
    int cur = s_cur, level = s_level, curmin = s_curmin;
    long long vis = s_vis;
    {
        const QEnt *qc = (level & 1) ? q1 : q0;
        for (int i = tid; i < cur; i += kBfsSmallThreads) sq[0][i] = qc[i];
    }
    int c = 0, p = 0;
    int w0 = 0, nw = 0, e0 = 0, e1 = 0;   // empty window: everything takes the global path
    int pmax = -1;
    bool finished = false;
    __syncthreads();

    // moves the window (all threads): the old one is written back, then rows
    // [base, base + rows) are read and the part whose entries fit is kept
    auto slide = [&](const WinPlan wp) {
        for (int i = tid; i < nw; i += kBfsSmallThreads)
            if (w_dist[i] >= 0) astore_i32(&dist[w0 + i], w_dist[i]);
        if (tid == 0) s_fit = 0;
        const int mode = wp.mode, nb0 = wp.base, rows = wp.rows;
        __syncthreads();
        for (int i = tid; i <= rows; i += kBfsSmallThreads) w_rp[i] = rp[nb0 + i];
        __syncthreads();
        // w_rp is non-decreasing: the fitting rows are a prefix (mode 1)
        // or a suffix (mode 2) of the rows read, so their count gives both
        // the window's size and its first row (one atomic per wave)
        {
            int cntl = 0;
            for (int i = tid; i <= rows; i += kBfsSmallThreads)
                cntl += (mode == 1 ? w_rp[i] - w_rp[0] : w_rp[rows] - w_rp[i]) <= kWinEntries ? 1 : 0;
            for (int o = 32; o > 0; o >>= 1) cntl += __shfl_xor(cntl, o, 64);
            if ((tid & 63) == 0 && cntl) atomicAdd(&s_fit, cntl);
        }
        __syncthreads();
        const int cnt = s_fit;   // >= 1: the first (mode 1) or last (mode 2) row always fits
        const int fit = cnt - 1;
        const int a = mode == 1 ? 0 : rows + 1 - cnt;
        if (a > 0) {   // move the kept row pointers to the front
            constexpr int kMv = (kWinRows + kBfsSmallThreads) / kBfsSmallThreads;   // >= (kWinRows + 1) / threads
            int tv[kMv];
#pragma unroll
            for (int r = 0; r < kMv; ++r) {
                const int i = tid + r * kBfsSmallThreads;
                tv[r] = i <= fit ? w_rp[a + i] : 0;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kMv; ++r) {
                const int i = tid + r * kBfsSmallThreads;
                if (i <= fit) w_rp[i] = tv[r];
            }
            __syncthreads();
        }
        w0 = nb0 + a;
        nw = fit;
        e0 = w_rp[0];
        e1 = w_rp[fit];
        for (int i = tid; i < e1 - e0; i += kBfsSmallThreads) w_col[i] = col[e0 + i];
        for (int i = tid; i < fit; i += kBfsSmallThreads) w_dist[i] = atomic_load_i32(&dist[w0 + i]);
        __syncthreads();
    };

    // bit-parallel levels from the current frontier (level `level`, all of it
    // and its neighbours inside the window); block-wide, returns kBitDone or
    // kBitMove with the state of the last frontier in b_*
    auto bit_levels = [&]() -> int {
        const int wv = tid >> 6, ln = tid & 63;
        // row masks and the frontier / visited words: one wave per 64 rows
        // (two words)
        for (int g = wv; g < kBitWords / 2; g += kBfsSmallThreads / 64) {
            const int r = g * 64 + ln;
            unsigned lo = 0u, hi = 0u;   // bit d: an entry at offset -d / +d
            bool f = false, v = false;
            if (r < nw) {
                const int row = w0 + r;
                const int j1 = w_rp[r + 1] - e0;
                for (int j = w_rp[r] - e0; j < j1; ++j) {
                    const int o = w_col[j] - row;
                    if (o < 0 && o >= -kBitBand) lo |= 1u << (-o);
                    else if (o > 0 && o <= kBitBand) hi |= 1u << o;
                }
                const int dd = w_dist[r];
                f = dd == level;
                v = dd >= 0;
            }
            for (int d = 1; d <= kBitBand; ++d) {
                const unsigned long long ml = __ballot((lo >> d) & 1u), mh = __ballot((hi >> d) & 1u);
                if (ln == 0) {
                    b_mp[d][2 * g] = (uint32_t)ml;
                    b_mp[d][2 * g + 1] = (uint32_t)(ml >> 32);
                    b_mm[d][2 * g] = (uint32_t)mh;
                    b_mm[d][2 * g + 1] = (uint32_t)(mh >> 32);
                }
            }
            const unsigned long long mf = __ballot(f), mv = __ballot(v);
            if (ln == 0) {
                b_f[2 * g] = (uint32_t)mf;
                b_f[2 * g + 1] = (uint32_t)(mf >> 32);
                b_v[2 * g] = (uint32_t)mv;
                b_v[2 * g + 1] = (uint32_t)(mv >> 32);
            }
        }
        if (tid == 0) b_app = 0;
        __syncthreads();
        // wave 0's state survives the flush rounds
        uint32_t mp[kBitBand + 1], mm[kBitBand + 1];
        uint32_t F = 0u, V = 0u, Fp = 0u, zone = 0u;
        int lev = level, pf0 = 0, pv0 = 0;
        if (wv == 0) {
            const int lane = ln;
#pragma unroll
            for (int d = 1; d <= kBitBand; ++d) {
                mp[d] = b_mp[d][lane];
                mm[d] = b_mm[d][lane];
            }
            F = b_f[lane];
            V = b_v[lane];
            pf0 = wave_sum_i(__popc(F));
            pv0 = wave_sum_i(__popc(V));
            // rows within band of an edge of the window that is not an edge of the graph
            const int lo_end = w0 > 0 ? band : 0;                 // rows [0, lo_end)
            const int hi_beg = w0 + nw < n ? nw - band : nw;      // rows [hi_beg, nw)
            for (int i = 0; i < 32; ++i) {
                const int r = lane * 32 + i;
                if (r < nw && (r < lo_end || r >= hi_beg)) zone |= 1u << i;
            }
        }
        int code;
        for (;;) {   // flush rounds
            if (wv == 0) {
                const int lane = ln;
                b_vs[lane] = V;   // visited before this round
                const int base = lev;
                int used = 0;
                for (;;) {
                    uint32_t fl = __shfl_up(F, 1, 64), fr = __shfl_down(F, 1, 64);
                    if (lane == 0) fl = 0u;
                    if (lane == 63) fr = 0u;
                    // every offset up to kBitBand: the masks of offsets the
                    // matrix does not use are zero (no branch per offset).  up:
                    // bit u from bit u - d (the words F:fl shifted), dn: bit u
                    // from bit u + d.
                    uint32_t N = 0u;
#pragma unroll
                    for (int d = 1; d <= kBitBand; ++d) {
                        const uint32_t up = __builtin_amdgcn_alignbit(F, fl, 32 - d);
                        const uint32_t dn = __builtin_amdgcn_alignbit(fr, F, d);
                        N = (up & mp[d]) | N;
                        N = (dn & mm[d]) | N;
                    }
                    const uint32_t nb = N & ~V;
                    if (!__any(nb != 0u)) {
                        code = kBitDone;
                        break;
                    }
                    V |= nb;
                    Fp = F;
                    F = nb;
                    ++lev;
                    b_ring[used][lane] = nb;
                    ++used;
                    if (__any((nb & zone) != 0u)) {
                        code = kBitMove;
                        break;
                    }
                    if (used == kBitRing) {
                        code = kBitFlush;
                        break;
                    }
                }
                b_v[lane] = V;
                if (lane == 0) {
                    b_code = code;
                    b_used = used;
                    b_base = base;
                }
            }
            __syncthreads();
            // ring -> distances: a thread per newly visited row
            {
                const int used = b_used, base = b_base;
                for (int r = tid; r < nw; r += kBfsSmallThreads) {
                    const int w = r >> 5;
                    const uint32_t bit = 1u << (r & 31);
                    if (!(b_v[w] & bit) || (b_vs[w] & bit)) continue;
                    for (int t = 0; t < used; t += 8) {
                        uint32_t x[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) x[i] = t + i < used ? b_ring[t + i][w] : 0u;
                        int hit = -1;
#pragma unroll
                        for (int i = 7; i >= 0; --i)
                            if (x[i] & bit) hit = i;
                        if (hit >= 0) {
                            w_dist[r] = base + t + hit + 1;
                            break;
                        }
                    }
                }
            }
            const int c_ = b_code;
            __syncthreads();   // the ring is read before the wave writes it again
            if (c_ != kBitFlush) break;
        }
        if (wv == 0) {
            const int lane = ln;
            code = b_code;
            const int pf = wave_sum_i(__popc(F));
            const int pv = wave_sum_i(__popc(V));
            const int fmin = wave_min_i(F ? lane * 32 + __ffs((int)F) - 1 : kIntMax);
            const int fmax = wave_max_i(F ? lane * 32 + 31 - __clz((int)F) : -1);
            const int pmx = wave_max_i(Fp ? lane * 32 + 31 - __clz((int)Fp) : -1);
            b_f[lane] = F;
            if (lane == 0) {
                b_level = lev;
                b_fmin = fmin;
                b_fmax = fmax;
                b_pmax = pmx;
                b_cnt = pf;
                // frontiers expanded here: the first one and every later one but
                // an unexpanded last (visited grows by the new vertices)
                b_vis = (long long)(pv - pv0) + pf0 - (code == kBitDone ? 0 : pf);
            }
        }
        __syncthreads();
        code = b_code;
        level = b_level;
        vis += b_vis;
        curmin = w0 + b_fmin;
        if (code == kBitDone) return code;
        // the new frontier into the queue (any order: distances are unique)
        cur = b_cnt;
        for (int r = tid; r < nw; r += kBfsSmallThreads) {
            if ((b_f[r >> 5] >> (r & 31)) & 1u) {
                const int pos = atomicAdd(&b_app, 1);
                sq[c ^ 1][pos] = QEnt{w_rp[r], w_rp[r + 1]};
            }
        }
        c ^= 1;
        __syncthreads();
        return code;
    };

    // every iteration expands one level, or a run of bit-parallel levels; at
    // most n levels exist
    for (;;) {
        if (band <= kBitBand && nw > 0 && pmax >= 0 && (w0 == 0 || curmin - band >= w0) &&
            (w0 + nw == n || (long long)pmax + band < (long long)w0 + nw)) {
            const int code = bit_levels();
            if (code == kBitDone) {
                finished = true;
                break;
            }
            if (cur > small_max) {   // hand over: the multi-block kernel reads the global queue
                QEnt *qc = (level & 1) ? q1 : q0;
                for (int i = tid; i < cur && i < kBfsSmallCap; i += kBfsSmallThreads) qc[i] = sq[c][i];
                break;
            }
            const int fmax = w0 + b_fmax, prev = b_pmax >= 0 ? w0 + b_pmax : -1;
            const WinPlan wp = plan_window(curmin, fmax, prev, band, n, w0, nw);
            pmax = fmax;
            if (wp.mode) slide(wp);
            continue;
        }
        const int pn = p == 2 ? 0 : p + 1;
        if (tid == 0) {   // the slot of the next level, last read two levels ago
            s_cnt[pn] = 0;
            s_min[pn] = kIntMax;
            s_max[pn] = -1;
        }
        QEnt *qn = (level & 1) ? q0 : q1;
        const int work = cur * lanes;
        // claims v for the next level; the window part touches LDS only, and
        // the next frontier is kept in LDS (global queue only past its size)
        auto visit = [&](int v) {
            if ((unsigned)v >= (unsigned)n) return;
            const int wv = v - w0;
            bool got;
            QEnt nv;
            if ((unsigned)wv < (unsigned)nw) {
                // in LDS the claim itself is the test (no separate read first)
                nv = QEnt{w_rp[wv], w_rp[wv + 1]};
                got = atomicCAS(&w_dist[wv], -1, level + 1) == -1;
            } else {
                if (dist[v] >= 0) return;
                nv = QEnt{rp[v], rp[v + 1]};
                got = atomicCAS(&dist[v], -1, level + 1) == -1;
            }
            if (got) {
                const int pos = atomicAdd(&s_cnt[p], 1);
                if (pos < kBfsSmallCap) sq[c ^ 1][pos] = nv;
                else qn[pos] = nv;
                atomicMin(&s_min[p], v);
                atomicMax(&s_max[p], v);
            }
        };
        for (int w = tid; w < work; w += kBfsSmallThreads) {
            const int f = w >> lsh, l = w & (lanes - 1);
            const QEnt u = sq[c][f];
            if (u.b >= e0 && u.e <= e1) {   // the row's columns are in the window
                for (int j = u.b + l; j < u.e; j += lanes) visit(w_col[j - e0]);
            } else {
                for (int j = u.b + l; j < u.e; j += lanes) visit(col[j]);
            }
        }
        __syncthreads();
        const int nxt = s_cnt[p], mn = s_min[p], mx = s_max[p];
        vis += cur;
        if (nxt == 0) {
            finished = true;
            break;
        }
        ++level;
        cur = nxt;
        curmin = mn;
        c ^= 1;
        p = pn;
        if (cur > small_max) {   // hand over: the multi-block kernel reads the global queue
            QEnt *qc = (level & 1) ? q1 : q0;
            for (int i = tid; i < cur && i < kBfsSmallCap; i += kBfsSmallThreads) qc[i] = sq[c][i];
            break;
        }
        const WinPlan wp = plan_window(mn, mx, pmax, band, n, w0, nw);
        pmax = mx;
        if (wp.mode) slide(wp);
    }
    // the window's distances go back to global memory before anyone reads them
    for (int i = tid; i < nw; i += kBfsSmallThreads)
        if (w_dist[i] >= 0) astore_i32(&dist[w0 + i], w_dist[i]);
    if (tid == 0) {
        st->bfs_visited = vis;
        if (finished) {
            st->bfs_done = 1;
            st->bfs_ecc = level;
            st->bfs_far = curmin;
        } else {
            st->bfs_cnt[level & 3] = cur;
            st->bfs_min[level & 3] = curmin;
            st->bfs_cnt[(level + 1) & 3] = 0;
            st->bfs_min[(level + 1) & 3] = kIntMax;
            st->bfs_lv[(k + 1) & 1] = level;
        }
    }
}

// ----------------------------------------------------- multi-block level --


// One level, top-down.  `lanes` consecutive lanes share a frontier vertex
// and take its neighbours in parallel (lane l: entries l, l + lanes, ...).
// Each thread takes kBfsItems work items at once and issues their loads
// together.  The queue holds row ranges, and the first batch's queue entries
// are read from both queues before the level is known, so a level costs four
// dependent memory round trips: (state, queue entry), column, claim
// (compare-and-swap on the distance, with the claimed vertex's row range
// loaded beside it), append.  Appends and the next frontier's minimum are
// aggregated per block -- one atomic on the shared counter per block and
// step, not per wave: all blocks append to the same counter, and same-address
// atomics serialise.  Block 0 retires the level and clears the counters of
// the level after next.
constexpr int kBfsItems = 4;

// A level whose frontier holds at least 1/kBottomUp of the vertices is
// expanded bottom-up: every unvisited vertex scans its row for a neighbour at
// the current level and stops at the first.  On a low-diameter graph (the
// Erdos-Renyi one) the middle levels reach most vertices, and there this
// reads a few entries per unvisited vertex where top-down would try every
// edge of the frontier with an atomic.  The decision uses only the level's
// size, which is final when the launch starts, so every block takes it alike.
// Distances are unique, so the result does not depend on the direction.
constexpr int kBottomUp = 8;

__global__ void __launch_bounds__(kBlock)
k_bfs_level(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *dist,
            QEnt *q0, QEnt *q1, int32_t n, int32_t lanes, int32_t k, int32_t precheck, DevState *st)
{
    __shared__ int s_cnt[kBlock / 64], s_base, s_steps, s_min;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lsh = __ffs(lanes) - 1;   // lanes is a power of two
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t span = stride * kBfsItems;
    const int64_t wbase0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63);
    QEnt pa[kBfsItems], pb[kBfsItems];   // first batch from queue 0 and queue 1
#pragma unroll
    for (int i = 0; i < kBfsItems; ++i) {
        const int64_t f = (wbase0 + i * stride + lane) >> lsh;
        pa[i] = QEnt{0, 0};
        pb[i] = QEnt{0, 0};
        if (f < n) {
            pa[i] = q0[f];
            pb[i] = q1[f];
        }
    }
    if (st->bfs_done) return;
    const int L = st->bfs_lv[k & 1];
    const int cur = min(st->bfs_cnt[L & 3], n);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (cur == 0) {
            bfs_finish(st, L);
        } else {
            st->bfs_visited += cur;
            st->bfs_lv[(k + 1) & 1] = L + 1;
            st->bfs_cnt[(L + 2) & 3] = 0;
            st->bfs_min[(L + 2) & 3] = kIntMax;
        }
    }
    if (cur == 0) return;
    const QEnt *qc = (L & 1) ? q1 : q0;
    QEnt *qn = (L & 1) ? q0 : q1;
    int *cnt_next = &st->bfs_cnt[(L + 1) & 3];
    const unsigned long long lt = (1ull << lane) - 1ull;
    int wmin = kIntMax;
    if ((int64_t)cur * kBottomUp >= n) {
        if (threadIdx.x == 0) s_min = kIntMax;
        // the vertex loop is uniform over the block (its waves meet at barriers)
        for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
            const int64_t vv = base + threadIdx.x;
            bool found = false;
            QEnt nv{0, 0};
            if (vv < n && dist[vv] < 0) {
                const int b = rp[vv], e = rp[vv + 1];
                for (int j = b; j < e; ++j) {
                    const int u = col[j];
                    if ((unsigned)u < (unsigned)n && dist[u] == L) {
                        found = true;
                        break;
                    }
                }
                if (found) {
                    dist[vv] = L + 1;   // only this thread writes vv; readers here compare with L
                    nv = QEnt{b, e};
                }
            }
            const unsigned long long m = __ballot(found);
            if (lane == 0) s_cnt[wv] = __popcll(m);
            __syncthreads();
            if (threadIdx.x == 0) {
                int sum = 0;
                for (int w = 0; w < kBlock / 64; ++w) {
                    const int c = s_cnt[w];
                    s_cnt[w] = sum;
                    sum += c;
                }
                s_base = sum > 0 ? atomicAdd(cnt_next, sum) : 0;
            }
            __syncthreads();
            if (found) {
                qn[s_base + s_cnt[wv] + __popcll(m & lt)] = nv;
                wmin = wmin < (int)vv ? wmin : (int)vv;
            }
            __syncthreads();   // s_cnt and s_base are reused by the next step
        }
        wmin = wave_min_i(wmin);
        if (lane == 0 && wmin != kIntMax) atomicMin(&s_min, wmin);
        __syncthreads();
        if (threadIdx.x == 0 && s_min != kIntMax) atomicMin(&st->bfs_min[(L + 1) & 3], s_min);
        return;
    }
    const int64_t items = (int64_t)cur * lanes;
    if (threadIdx.x == 0) s_min = kIntMax;
    // the batch loop is uniform over the block (its waves meet at barriers)
    const int64_t bbase0 = (int64_t)blockIdx.x * kBlock;
    bool first = true;
    for (int64_t bbase = bbase0; bbase < items; bbase += span, first = false) {
        const int64_t wbase = bbase + (threadIdx.x & ~63);
        int j[kBfsItems], e[kBfsItems];
#pragma unroll
        for (int i = 0; i < kBfsItems; ++i) {
            const int64_t w = wbase + i * stride + lane;
            QEnt u{0, 0};
            if (w < items) u = first ? ((L & 1) ? pb[i] : pa[i]) : qc[(int)(w >> lsh)];
            j[i] = u.b + (int)(w & (lanes - 1));
            e[i] = w < items ? u.e : 0;
        }
        int steps = 0;
#pragma unroll
        for (int i = 0; i < kBfsItems; ++i) {
            const int si = j[i] < e[i] ? (e[i] - j[i] + lanes - 1) >> lsh : 0;
            steps = steps > si ? steps : si;
        }
        steps = wave_max_i(steps);
        if (threadIdx.x == 0) s_steps = 0;
        __syncthreads();
        if (lane == 0) atomicMax(&s_steps, steps);
        __syncthreads();
        steps = s_steps;
        __syncthreads();   // everyone has read s_steps before the next batch resets it
        for (int t = 0; t < steps; ++t) {
            int v[kBfsItems];
            bool found[kBfsItems];
            QEnt nv[kBfsItems];
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                v[i] = j[i] < e[i] ? col[j[i]] : -1;
                if ((unsigned)v[i] >= (unsigned)n) v[i] = -1;
                j[i] += lanes;
            }
            if (precheck) {
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i)
                    if (v[i] >= 0 && dist[v[i]] >= 0) v[i] = -1;
            }
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                nv[i] = QEnt{0, 0};
                if (v[i] >= 0) nv[i] = QEnt{rp[v[i]], rp[v[i] + 1]};
            }
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i)   // self-loops fail here: the vertex being expanded is visited
                found[i] = v[i] >= 0 && atomicCAS(&dist[v[i]], -1, L + 1) == -1;
            unsigned long long m[kBfsItems];
            int total = 0;
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                m[i] = __ballot(found[i]);
                total += __popcll(m[i]);
            }
            // block aggregation: one atomic on the shared counter per block and step
            if (lane == 0) s_cnt[wv] = total;
            __syncthreads();
            if (threadIdx.x == 0) {
                int sum = 0;
                for (int w = 0; w < kBlock / 64; ++w) {
                    const int c = s_cnt[w];
                    s_cnt[w] = sum;
                    sum += c;
                }
                s_base = sum > 0 ? atomicAdd(cnt_next, sum) : 0;
            }
            __syncthreads();
            int base = s_base + s_cnt[wv];
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                if (found[i]) {
                    qn[base + __popcll(m[i] & lt)] = nv[i];
                    wmin = wmin < v[i] ? wmin : v[i];
                }
                base += __popcll(m[i]);
            }
            __syncthreads();   // s_cnt and s_base are reused by the next step
        }
    }
    wmin = wave_min_i(wmin);
    if (lane == 0 && wmin != kIntMax) atomicMin(&s_min, wmin);
    __syncthreads();
    if (threadIdx.x == 0 && s_min != kIntMax) atomicMin(&st->bfs_min[(L + 1) & 3], s_min);
}

// ------------------------------------------------ persistent large levels --
//
// Expands every level whose frontier is larger than small_max in ONE launch:
// the blocks meet at a grid barrier between levels instead of ending the
// kernel.  Data other blocks produce within the launch (queue entries, level
// counters, the barrier count) is written and read with agent-scope atomics,
// and the barrier orders them with agent-scope release and acquire fences
// (the HIP memory model's guarantee, not a property of one chip).  The read-only CSR pattern and the
// distance pre-check use plain loads (a stale distance only costs a failing
// compare-and-swap).  Every wait is bounded; if one runs out the kernel
// raises st->guard and the host repeats the BFS with one launch per level.
// The grid is small, so its blocks can all be resident next to other work.

__device__ inline int aload(const int32_t *p)
{
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void astore(int32_t *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline QEnt aload_q(const QEnt *p)
{
    const uint64_t v = __hip_atomic_load(reinterpret_cast<uint64_t *>(const_cast<QEnt *>(p)), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return QEnt{(int32_t)(uint32_t)(v & 0xffffffffull), (int32_t)(uint32_t)(v >> 32)};
}
__device__ inline void astore_q(QEnt *p, QEnt q)
{
    const uint64_t v = (uint64_t)(uint32_t)q.b | ((uint64_t)(uint32_t)q.e << 32);
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kBarSpinLimit = 1u << 22;

__global__ void __launch_bounds__(kBlock)
k_bfs_persist(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t *dist, QEnt *q0,
              QEnt *q1, int32_t n, int32_t lanes, int32_t small_max, int32_t k, DevState *st)
{
    __shared__ int s_ok, s_cnt[kBlock / 64], s_base, s_steps, s_min;
    if (aload(&st->bfs_done)) return;
    int L = aload(&st->bfs_lv[k & 1]);
    int cur = aload(&st->bfs_cnt[L & 3]);
    const bool b0 = blockIdx.x == 0 && threadIdx.x == 0;
    if (cur <= small_max) {   // nothing large to do: hand the level on
        if (b0) astore(&st->bfs_lv[(k + 1) & 1], L);
        return;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lsh = __ffs(lanes) - 1;   // lanes is a power of two
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t span = stride * kBfsItems;
    long long visited = 0;
    for (uint32_t round = 1;; ++round) {
        if (b0) {
            visited += cur;
            astore(&st->bfs_cnt[(L + 2) & 3], 0);
            astore(&st->bfs_min[(L + 2) & 3], kIntMax);
        }
        const QEnt *qc = (L & 1) ? q1 : q0;
        QEnt *qn = (L & 1) ? q0 : q1;
        int *cnt_next = &st->bfs_cnt[(L + 1) & 3];
        int wmin = kIntMax;
        const int64_t items = (int64_t)min(cur, n) * lanes;
        if (threadIdx.x == 0) s_min = kIntMax;
        for (int64_t bbase = (int64_t)blockIdx.x * kBlock; bbase < items; bbase += span) {   // block-uniform
            const int64_t wbase = bbase + (threadIdx.x & ~63);
            int j[kBfsItems], e[kBfsItems];
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                const int64_t w = wbase + i * stride + lane;
                const QEnt u = w < items ? aload_q(&qc[(int)(w >> lsh)]) : QEnt{0, 0};
                j[i] = u.b + (int)(w & (lanes - 1));
                e[i] = w < items ? u.e : 0;
            }
            int steps = 0;
#pragma unroll
            for (int i = 0; i < kBfsItems; ++i) {
                const int si = j[i] < e[i] ? (e[i] - j[i] + lanes - 1) >> lsh : 0;
                steps = steps > si ? steps : si;
            }
            steps = wave_max_i(steps);
            if (threadIdx.x == 0) s_steps = 0;
            __syncthreads();
            if (lane == 0) atomicMax(&s_steps, steps);
            __syncthreads();
            steps = s_steps;
            __syncthreads();
            for (int t = 0; t < steps; ++t) {
                int v[kBfsItems];
                bool found[kBfsItems];
                QEnt nv[kBfsItems];
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i) {
                    v[i] = j[i] < e[i] ? col[j[i]] : -1;
                    if ((unsigned)v[i] >= (unsigned)n) v[i] = -1;
                    j[i] += lanes;
                }
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i) {
                    nv[i] = QEnt{0, 0};
                    if (v[i] >= 0) nv[i] = QEnt{rp[v[i]], rp[v[i] + 1]};
                }
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i)
                    found[i] = v[i] >= 0 && atomicCAS(&dist[v[i]], -1, L + 1) == -1;
                unsigned long long m[kBfsItems];
                int total = 0;
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i) {
                    m[i] = __ballot(found[i]);
                    total += __popcll(m[i]);
                }
                if (lane == 0) s_cnt[wv] = total;
                __syncthreads();
                if (threadIdx.x == 0) {
                    int sum = 0;
                    for (int w = 0; w < kBlock / 64; ++w) {
                        const int c = s_cnt[w];
                        s_cnt[w] = sum;
                        sum += c;
                    }
                    s_base = sum > 0 ? atomicAdd(cnt_next, sum) : 0;
                }
                __syncthreads();
                int base = s_base + s_cnt[wv];
#pragma unroll
                for (int i = 0; i < kBfsItems; ++i) {
                    if (found[i]) {
                        astore_q(&qn[base + __popcll(m[i] & lt)], nv[i]);
                        wmin = wmin < v[i] ? wmin : v[i];
                    }
                    base += __popcll(m[i]);
                }
                __syncthreads();
            }
        }
        wmin = wave_min_i(wmin);
        if (lane == 0 && wmin != kIntMax) atomicMin(&s_min, wmin);
        __syncthreads();
        if (threadIdx.x == 0 && s_min != kIntMax) atomicMin(&st->bfs_min[(L + 1) & 3], s_min);
        // Grid barrier.  Every thread's stores and claims of this level are
        // released at agent scope before its block arrives; the arrival is a
        // release read-modify-write, the wait ends with an acquire fence, and
        // every thread acquires at agent scope after it, so the next level
        // reads what all blocks wrote in this one.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            s_ok = 1;
            __hip_atomic_fetch_add(&st->bfs_bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = round * gridDim.x;
            uint32_t spins = 0;
            while (__hip_atomic_load(&st->bfs_bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kBarSpinLimit) {
                    s_ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // pairs with the arrivals' release
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!s_ok) {
            if (threadIdx.x == 0) atomicOr(&st->guard, 1);
            return;
        }
        const int nxt = aload(cnt_next);
        if (nxt == 0) {   // level L was the last non-empty one
            if (b0) {
                st->bfs_visited += visited;
                astore(&st->bfs_ecc, L);
                astore(&st->bfs_far, aload(&st->bfs_min[L & 3]));
                astore(&st->bfs_done, 1);
            }
            return;
        }
        L += 1;
        cur = nxt;
        if (cur <= small_max) {
            if (b0) {
                st->bfs_visited += visited;
                astore(&st->bfs_lv[(k + 1) & 1], L);
            }
            return;
        }
    }
}

int launch_bfs_round(hipStream_t s, const BfsBufs &b, int levels, int k)
{
    if (b.persist) {
        hipLaunchKernelGGL(k_bfs_small, dim3(1), dim3(kBfsSmallThreads), 0, s, b.rp, b.col, b.dist, b.q0,
                           b.q1, b.n, b.lanes, b.small_max, b.band, k, b.st);
        ++k;
        int grid = (b.n + kBlock - 1) / kBlock;
        if (grid > b.grid) grid = b.grid;
        hipLaunchKernelGGL(k_bfs_persist, dim3(grid), dim3(kBlock), 0, s, b.rp, b.col, b.dist, b.q0, b.q1, b.n,
                           b.lanes, b.small_max, k, b.st);
        return k + 1;
    }

    hipLaunchKernelGGL(k_bfs_small, dim3(1), dim3(kBfsSmallThreads), 0, s, b.rp, b.col, b.dist, b.q0,
                       b.q1, b.n, b.lanes, b.small_max, b.band, k, b.st);
    ++k;
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > b.grid) grid = b.grid;
    for (int l = 0; l < levels; ++l, ++k)
        hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(kBlock), 0, s, b.rp, b.col, b.dist, b.q0, b.q1,
                           b.n, b.lanes, k, b.precheck, b.st);
    return k;
}

// ------------------------------------------------ distance histogram --

// hist[d] += #{v : dist[v] = d}, d >= 1 (unreached vertices and the source are
// skipped).  Distances below kHistLds are counted in LDS first.
constexpr int kHistLds = 2048;

__global__ void __launch_bounds__(kBlock)
k_dist_hist(const int32_t *__restrict__ dist, int32_t n, unsigned long long *hist)
{
    __shared__ unsigned int lh[kHistLds];
    for (int i = threadIdx.x; i < kHistLds; i += kBlock) lh[i] = 0u;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int d = dist[v];
        if (d < 1) continue;
        if (d < kHistLds) atomicAdd(&lh[d], 1u);
        else atomicAdd(&hist[d], 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistLds; i += kBlock)
        if (lh[i]) atomicAdd(&hist[i], (unsigned long long)lh[i]);
}

void launch_dist_hist(hipStream_t s, const int32_t *dist, int32_t n, unsigned long long *hist)
{
    int grid = (n + kBlock - 1) / kBlock;
    if (grid > 1024) grid = 1024;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_dist_hist, dim3(grid), dim3(kBlock), 0, s, dist, n, hist);
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
__global__ void k_bfs_seed_roots(const int32_t *rp, const int32_t *label, int32_t *dist, QEnt *q0,
                                 unsigned long long *best, int32_t n, DevState *st)
{
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const bool root = label[v] == v;
        dist[v] = root ? 0 : -1;
        if (root) {
            best[v] = 0ull;
            const int pos = atomicAdd(&st->bfs_cnt[0], 1);
            q0[pos] = QEnt{rp[v], rp[v + 1]};
        }
    }
}

// The sources were appended to bfs_cnt[0]; their smallest vertex is not
// needed (components take their own argmax).
__global__ void k_bfs_seed_finish(DevState *st, int roots)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int cnt = st->bfs_cnt[0];
        bfs_start(st, cnt, 0);
        if (roots) {
            st->ncomp = cnt;
            st->comp_best = 0ull;
        }
    }
}

__global__ void k_zero_sources(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->bfs_cnt[0] = 0;
}

void launch_bfs_seed_roots(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_zero_sources, dim3(1), dim3(64), 0, s, b.st);
    hipLaunchKernelGGL(k_bfs_seed_roots, dim3(grid), dim3(kBlock), 0, s, b.rp, b.label, b.dist, b.q0, b.best,
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
__global__ void k_bfs_seed_far(const int32_t *rp, const int32_t *label, int32_t *dist, QEnt *q0, int32_t *tarr,
                               unsigned long long *best, int32_t n, DevState *st)
{
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        if (label[v] == v) {
            const int t = (int)(0xffffffffu - (unsigned)(best[v] & 0xffffffffull));
            tarr[v] = t;
            best[v] = 0ull;
            dist[t] = 0;
            const int pos = atomicAdd(&st->bfs_cnt[0], 1);
            q0[pos] = QEnt{rp[t], rp[t + 1]};
        }
    }
}

void launch_bfs_seed_far(hipStream_t s, const BfsBufs &b)
{
    int grid = (b.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    launch_fill_i32(s, b.dist, b.n, -1);
    hipLaunchKernelGGL(k_zero_sources, dim3(1), dim3(64), 0, s, b.st);
    hipLaunchKernelGGL(k_bfs_seed_far, dim3(grid), dim3(kBlock), 0, s, b.rp, b.label, b.dist, b.q0, b.tarr,
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


// ------------------------------------- bit-parallel levels over diagonals --
//
// When the stored pattern lies on at most kDiaMax diagonals (offsets j - i),
// as grids and bands do, a level can be formed on bit vectors of all n rows
// instead of a queue: v is at the next level iff it is unvisited and, for
// some offset d, u = v - d is in the frontier and row u stores column v.  The
// masks are kept aligned to v (bit v of mask t: row v - d_t stores column v),
// so each thread forms one 32-bit word of the next frontier from one mask
// word and one 32-bit window of the frontier per diagonal (a funnel shift of
// two words, one word when d_t is a multiple of 32), removes the visited
// bits, writes the new vertices' distances, and its block adds the count of
// new vertices and their smallest index to the level state.  Launch k expands
// level k (a sweep runs one level per launch from k = 0), so the buffers are
// chosen without reading the state; block 0 keeps the level-state protocol of
// the queue kernels (retire level k, or finish when it is empty), so the
// stop, the eccentricity, the farthest vertex (smallest index of the last
// level) and the distances are the queue kernels' integers.  Once a level is
// empty every later launch reads an empty frontier and writes nothing but
// zero words.

// Distinct nonzero offsets of the stored entries into st->dia_off (slots
// filled from 0; 0 marks an empty slot), or st->dia_over when there are more
// than kDiaMax.  One row per thread, its entries loaded together.
__global__ void __launch_bounds__(kBlock)
k_dia_offsets(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n, DevState *st)
{
    __shared__ int32_t tab[kDiaMax];
    __shared__ int over;
    if (threadIdx.x < kDiaMax) tab[threadIdx.x] = 0;
    if (threadIdx.x == 0) over = 0;
    __syncthreads();
    constexpr int kRow = 16;   // entries loaded at once
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < n && !*(volatile int *)&over;
         i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
        if (i >= n) continue;
        const int b = rp[i], e = rp[i + 1];
        for (int k0 = b; k0 < e; k0 += kRow) {
            int c[kRow];
#pragma unroll
            for (int j = 0; j < kRow; ++j) c[j] = k0 + j < e ? col[k0 + j] : (int)i;
#pragma unroll
            for (int j = 0; j < kRow; ++j) {
                if ((unsigned)c[j] >= (unsigned)n) continue;   // ignored, as by the queue kernels
                const int d = c[j] - (int)i;
                if (d == 0) continue;
                int t = 0;
                while (t < kDiaMax) {   // plain reads first: the offset is almost always known
                    const int v = tab[t];
                    if (v == d || v == 0) break;
                    ++t;
                }
                if (t < kDiaMax && tab[t] == d) continue;
                bool put = false;
                for (t = 0; t < kDiaMax && !put; ++t) {
                    const int old = atomicCAS(&tab[t], 0, d);
                    put = old == 0 || old == d;
                }
                if (!put) over = 1;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && over) atomicOr(&st->dia_over, 1);
    if (threadIdx.x < kDiaMax && !over) {
        const int d = tab[threadIdx.x];
        if (d != 0) {
            // most blocks find every offset already there: read the table
            // first (coherent loads) so that only new offsets take a CAS
            bool put = false;
            for (int t = 0; t < kDiaMax && !put; ++t) {
                const int v = __hip_atomic_load(&st->dia_off[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v == d) put = true;
                if (v == 0) break;
            }
            for (int t = 0; t < kDiaMax && !put; ++t) {
                const int old = atomicCAS(&st->dia_off[t], 0, d);
                put = old == 0 || old == d;
            }
            if (!put) atomicOr(&st->dia_over, 1);
        }
    }
}

__global__ void k_dia_reset(DevState *st)
{
    if (threadIdx.x < kDiaMax) st->dia_off[threadIdx.x] = 0;
    if (threadIdx.x == 0) st->dia_over = 0;
}

void launch_dia_detect(hipStream_t s, const BfsBufs &b)
{
    int g = (b.n + kBlock - 1) / kBlock;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_dia_reset, dim3(1), dim3(64), 0, s, b.st);
    hipLaunchKernelGGL(k_dia_offsets, dim3(g), dim3(kBlock), 0, s, b.rp, b.col, b.n, b.st);
}

// Row masks: bit u of raw[t] is set iff row u stores column u + d_t.  A wave
// covers 64 rows = two words of each mask and writes them alone.
__global__ void __launch_bounds__(kBlock)
k_dia_rowmasks(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n, int32_t nw,
               uint32_t *raw, DiaOffs o)
{
    const int lane = threadIdx.x & 63;
    constexpr int kRow = 16;
    // wave-uniform loop: a wave's lanes share the base row
    for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < n;
         base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + lane;
        uint32_t has = 0u;
        if (i < n) {
            const int b = rp[i], e = rp[i + 1];
            for (int k0 = b; k0 < e; k0 += kRow) {
                int c[kRow];
#pragma unroll
                for (int j = 0; j < kRow; ++j) c[j] = k0 + j < e ? col[k0 + j] : (int)i;
#pragma unroll
                for (int j = 0; j < kRow; ++j) {
                    if ((unsigned)c[j] >= (unsigned)n) continue;   // so every neighbour u + d is a row
                    const int d = c[j] - (int)i;
                    for (int t = 0; t < o.nd; ++t)
                        if (o.d[t] == d) has |= 1u << t;
                }
            }
        }
        const int w0 = (int)(base >> 5);
        for (int t = 0; t < o.nd; ++t) {
            const unsigned long long m = __ballot((has >> t) & 1u);
            if (lane == 0) {
                raw[(size_t)t * nw + w0] = (uint32_t)(m & 0xffffffffull);
                if (w0 + 1 < nw) raw[(size_t)t * nw + w0 + 1] = (uint32_t)(m >> 32);
            }
        }
    }
}

// 32 bits of bit vector B starting at bit position p (bits outside [0, 32 nw) read as 0).
__device__ inline uint32_t dia_window(const uint32_t *B, int64_t p, int32_t nw)
{
    const int64_t q = p >> 5;   // floor, also for p < 0
    const int r = (int)(p & 31);
    const uint32_t lo = (q >= 0 && q < nw) ? B[q] : 0u;
    if (r == 0) return lo;
    const uint32_t hi = (q + 1 >= 0 && q + 1 < nw) ? B[q + 1] : 0u;
    return (lo >> r) | (hi << (32 - r));
}

// The window of diagonal t at word w starts at bit 32 w - d_t = 32 (w + q_t) + r_t.
// F holds the words [lo, hi) of the bit vector (words outside [0, nw) read
// as 0; callers keep the words a window needs inside [lo, hi)).  Both words
// are loaded unconditionally from clamped indices, so a word's windows issue
// their loads together.
__device__ inline uint32_t dia_win(const uint32_t *F, int lo, int hi, int w, int qt, int rt, int32_t nw)
{
    const int q = w + qt;
    const int i0 = q < lo ? lo : (q >= hi ? hi - 1 : q);
    const int i1 = q + 1 < lo ? lo : (q + 1 >= hi ? hi - 1 : q + 1);
    uint32_t w0 = F[i0 - lo], w1 = F[i1 - lo];
    w0 = (q >= 0 && q < nw) ? w0 : 0u;
    w1 = (q + 1 >= 0 && q + 1 < nw) ? w1 : 0u;
    return __builtin_amdgcn_alignbit(w1, w0, rt);
}

// Aligned masks: word w of dm[t] = bits v in [32 w, 32 w + 32) of "row v - d_t
// stores column v" = the 32-bit window of raw[t] at 32 w - d_t.
__global__ void __launch_bounds__(kBlock)
k_dia_align(const uint32_t *__restrict__ raw, uint32_t *dm, int32_t nw, DiaOffs o)
{
    for (int w = blockIdx.x * kBlock + threadIdx.x; w < nw; w += gridDim.x * kBlock)
        for (int t = 0; t < o.nd; ++t)
            dm[(size_t)t * nw + w] = dia_window(raw + (size_t)t * nw, 32 * (int64_t)w - o.d[t], nw);
}

void launch_dia_masks(hipStream_t s, const BfsBufs &b)
{
    uint32_t *raw = b.draw;
    int g = (b.n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_dia_rowmasks, dim3(g), dim3(kBlock), 0, s, b.rp, b.col, b.n, b.nwords, raw, b.doff);
    int ga = (b.nwords + kBlock - 1) / kBlock;
    if (ga > 4096) ga = 4096;
    hipLaunchKernelGGL(k_dia_align, dim3(ga), dim3(kBlock), 0, s, raw, b.dm, b.nwords, b.doff);
}

// Both frontier buffers and the visited bits start empty.  The per-level
// kernel then writes only the words that gain vertices, so a buffer can keep
// bits of the frontier two (four, ...) levels back; those vertices are
// visited, and so are all their neighbours (a BFS neighbour is at most one
// level further), so the extra bits add only visited vertices, which the
// level removes -- the levels are exact, and a level dirties only the words
// of its own frontier.
__global__ void k_dia_clear(uint32_t *f0, uint32_t *f1, uint32_t *v, int32_t nw)
{
    for (int w = blockIdx.x * kBlock + threadIdx.x; w < nw; w += gridDim.x * kBlock) {
        f0[w] = 0u;
        f1[w] = 0u;
        v[w] = 0u;
    }
}

__global__ void k_dia_seed(uint32_t *f0, uint32_t *v, int32_t *dist, int32_t src, int32_t *pcnt, int32_t *pmin,
                           DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        f0[src >> 5] = 1u << (src & 31);
        v[src >> 5] = 1u << (src & 31);
        dist[src] = 0;
        bfs_start(st, 1, src);
        st->dia_base = 0;
    }
    // level 0's per-block partials (one-level kernel): the source alone
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kDiaPartMax; i += gridDim.x * blockDim.x) {
        pcnt[i] = i == 0 ? 1 : 0;
        pmin[i] = i == 0 ? src : kIntMax;
    }
}

void launch_dia_seed(hipStream_t s, const BfsBufs &b, int32_t src)
{
    int g = (b.nwords + kBlock - 1) / kBlock;
    if (g > 1024) g = 1024;
    launch_fill_i32(s, b.dist, b.n, -1);
    hipLaunchKernelGGL(k_dia_clear, dim3(g), dim3(kBlock), 0, s, b.df0, b.df1, b.dv, b.nwords);
    hipLaunchKernelGGL(k_dia_seed, dim3(1), dim3(kBlock), 0, s, b.df0, b.dv, b.dist, src, b.part_cnt, b.part_min,
                       b.st);
}

// Launch j of a round expands level L = st->dia_base + j; rounds are
// kDiaRound launches, and k_dia_round_end (the round's last launch) moves
// the base on, so every launch of a round has fixed arguments (the round can
// be replayed as a captured graph) and its frontier parity is j & 1.  Each
// block stores its count of new vertices and their smallest index in slot
// blockIdx.x of the partials of parity (L + 1) & 1 -- plain stores, no
// same-address atomics across the grid; wave 0 of block 0 in the next launch
// sums them (all loads at once) and retires the level: the level-state
// protocol of the queue kernels, with the sums in place of the counters.
template <int ND>
__global__ void __launch_bounds__(kBlock)
k_dia_level(const uint32_t *__restrict__ fc, uint32_t *__restrict__ fn, uint32_t *dv, const uint32_t *__restrict__ dm,
            int32_t *dist, int32_t nw, int32_t j, DiaOffs o, const int32_t *__restrict__ pc_cur,
            const int32_t *__restrict__ pm_cur, int32_t *pc_next, int32_t *pm_next, DevState *st)
{
    __shared__ int s_cnt[kBlock / 64], s_min[kBlock / 64];
    const int L = st->dia_base + j;   // needed only for the distances and the retirement
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        // level L's size and smallest vertex from the previous launch's
        // partials (the seed's for level 0), then its retirement
        const int lane = threadIdx.x;
        const int done = st->bfs_done;
        int c = 0, m = kIntMax;
        for (int i = lane; i < (int)gridDim.x; i += 64) {
            c += pc_cur[i];
            m = m < pm_cur[i] ? m : pm_cur[i];
        }
        c = wave_sum_i(c);
        m = wave_min_i(m);
        if (lane == 0 && !done) {
            if (c == 0) {
                st->bfs_done = 1;   // level L is empty: L - 1 was the last
                st->bfs_ecc = L - 1;
                st->bfs_far = st->bfs_min[(L - 1) & 3];
            } else {
                st->bfs_visited += c;
                st->bfs_min[L & 3] = m;
                st->bfs_lv[(L + 1) & 1] = L + 1;
            }
        }
    }
    // XCD-aware placement: the blocks of one XCD (blockIdx.x mod kNumXcd)
    // take consecutive 256-word chunks, so the frontier words a window reads
    // a few chunks away were mostly written on the same XCD
    const int G = gridDim.x, b = blockIdx.x;
    const int nx = G < kNumXcd ? G : kNumXcd, xq = G / nx, xr = G % nx, x = b % nx;
    const int chunk = x * xq + (x < xr ? x : xr) + b / nx;
    int cnt = 0, mn = kIntMax;
    for (int w = chunk * kBlock + threadIdx.x; w < nw; w += G * kBlock) {
        const uint32_t vis = dv[w];
        uint32_t nb = 0u;
#pragma unroll
        for (int t = 0; t < ND; ++t) nb |= dia_win(fc, 0, nw, w, o.q[t], o.r[t], nw) & dm[(size_t)t * nw + w];
        nb &= ~vis;
        if (nb) {   // words without new vertices keep older frontiers' bits: see k_dia_clear
            fn[w] = nb;
            dv[w] = vis | nb;
            cnt += __popc(nb);
            const int v0 = 32 * w + __ffs(nb) - 1;
            mn = mn < v0 ? mn : v0;
            for (uint32_t bb = nb; bb; bb &= bb - 1u) dist[32 * w + __ffs(bb) - 1] = L + 1;
        }
    }
    cnt = wave_sum_i(cnt);
    mn = wave_min_i(mn);
    if ((threadIdx.x & 63) == 0) {
        s_cnt[threadIdx.x >> 6] = cnt;
        s_min[threadIdx.x >> 6] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0, m = kIntMax;
        for (int i = 0; i < kBlock / 64; ++i) {
            c += s_cnt[i];
            m = m < s_min[i] ? m : s_min[i];
        }
        pc_next[blockIdx.x] = c;
        pm_next[blockIdx.x] = m;
    }
}

__global__ void k_dia_round_end(DevState *st, int32_t levels)
{
    if (threadIdx.x == 0) st->dia_base += levels;
}

// Two levels per launch.  A block takes a chunk of kBlock words (one per
// thread) and loads into LDS the level-L frontier over the chunk widened by
// 2R words on each side (R: the most words a diagonal's window reaches).  It
// forms the neighbours of that frontier at every word of the chunk widened
// by R -- the words the chunk's level-(L + 1) windows read -- and from those
// level L + 2 at its own words.  The neighbours are not stripped of visited
// vertices (other blocks update those words in this launch): besides level
// L + 1 they hold only vertices of levels L - 1 and L, whose neighbours are at
// most at level L + 1 and are removed at the thread's own word together with
// its visited bits and its exact level L + 1.  Launch j of a round expands
// levels L0 + 1 and L0 + 2, L0 = dia_base + 2 j, and writes per-block partials
// of both; wave 0 of block 0 of the next launch retires them (at L0 = 0 it
// counts the source).  Only words that gain vertices are written (see
// k_dia_clear).  LDS: (2 kBlock + 6 R) words.  (Staging the halo words'
// masks in LDS as well, or loading six words' masks at once into registers,
// measured slower at 128^3.)
template <int ND>
__global__ void __launch_bounds__(kBlock)
k_dia_level2(const uint32_t *__restrict__ fc, uint32_t *__restrict__ fn, uint32_t *dv, const uint32_t *__restrict__ dm,
             int32_t *dist, int32_t nw, int32_t j, int32_t R, DiaOffs o, const int32_t *__restrict__ pc_cur,
             const int32_t *__restrict__ pm_cur, int32_t *pc_next, int32_t *pm_next, DevState *st)
{
    extern __shared__ uint32_t lds[];
    __shared__ int s_cnt[2][kBlock / 64], s_min[2][kBlock / 64];
    const int L0 = st->dia_base + 2 * j;
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        // retire levels L0 - 1 and L0 (the previous launch's partials)
        const int lane = threadIdx.x;
        const int done = st->bfs_done;
        int ca = 0, ma = kIntMax, cb = 0, mb = kIntMax;
        if (L0 > 0)
            for (int i = lane; i < (int)gridDim.x; i += 64) {
                ca += pc_cur[i];
                ma = ma < pm_cur[i] ? ma : pm_cur[i];
                cb += pc_cur[kDiaPartMax + i];
                mb = mb < pm_cur[kDiaPartMax + i] ? mb : pm_cur[kDiaPartMax + i];
            }
        ca = wave_sum_i(ca);
        ma = wave_min_i(ma);
        cb = wave_sum_i(cb);
        mb = wave_min_i(mb);
        if (lane == 0 && !done) {
            if (L0 == 0) {
                st->bfs_visited += 1;   // the source (bfs_far already holds it)
            } else if (ca == 0) {       // level L0 - 1 empty: L0 - 2 was the last
                st->bfs_done = 1;
                st->bfs_ecc = L0 - 2;
            } else if (cb == 0) {       // level L0 empty: L0 - 1 was the last
                st->bfs_visited += ca;
                st->bfs_done = 1;
                st->bfs_ecc = L0 - 1;
                st->bfs_far = ma;
            } else {
                st->bfs_visited += ca + cb;
                st->bfs_far = mb;
                st->bfs_lv[0] = L0;
            }
        }
    }
    const int G = gridDim.x, b = blockIdx.x;
    const int nx = G < kNumXcd ? G : kNumXcd, xq = G / nx, xr = G % nx, x = b % nx;
    const int nchunks = (nw + kBlock - 1) / kBlock;
    const int NF = kBlock + 4 * R, NN = kBlock + 2 * R;
    uint32_t *LF = lds, *LN = lds + NF;   // level-L frontier from c0 - 2R, neighbours from c0 - R
    int c1 = 0, m1 = kIntMax, c2 = 0, m2 = kIntMax;
    for (int chunk = x * xq + (x < xr ? x : xr) + b / nx; chunk < nchunks; chunk += G) {
        const int c0 = chunk * kBlock;
        for (int i = threadIdx.x; i < NF; i += kBlock) {
            const int w = c0 - 2 * R + i;
            LF[i] = (w >= 0 && w < nw) ? fc[w] : 0u;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < NN; i += kBlock) {
            const int u = c0 - R + i;
            uint32_t nb = 0u;
            if (u >= 0 && u < nw) {
                const int iu = i + R;   // u's index in LF
#pragma unroll
                for (int t = 0; t < ND; ++t) {
                    const int k = iu + o.q[t];
                    nb |= __builtin_amdgcn_alignbit(LF[k + 1], LF[k], o.r[t]) & dm[(size_t)t * nw + u];
                }
            }
            LN[i] = nb;
        }
        __syncthreads();
        const int w = c0 + threadIdx.x;
        if (w < nw) {
            const uint32_t vis = dv[w];
            const int iw = threadIdx.x + R;   // w's index in LN
            const uint32_t own1 = LN[iw] & ~vis;
            uint32_t nb2 = 0u;
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                const int k = iw + o.q[t];
                nb2 |= __builtin_amdgcn_alignbit(LN[k + 1], LN[k], o.r[t]) & dm[(size_t)t * nw + w];
            }
            nb2 &= ~(vis | own1);
            if (nb2) fn[w] = nb2;
            if (own1 | nb2) dv[w] = vis | own1 | nb2;
            if (own1) {
                c1 += __popc(own1);
                const int v0 = 32 * w + __ffs(own1) - 1;
                m1 = m1 < v0 ? m1 : v0;
                for (uint32_t bb = own1; bb; bb &= bb - 1u) dist[32 * w + __ffs(bb) - 1] = L0 + 1;
            }
            if (nb2) {
                c2 += __popc(nb2);
                const int v0 = 32 * w + __ffs(nb2) - 1;
                m2 = m2 < v0 ? m2 : v0;
                for (uint32_t bb = nb2; bb; bb &= bb - 1u) dist[32 * w + __ffs(bb) - 1] = L0 + 2;
            }
        }
        __syncthreads();   // LDS reused by the next chunk
    }
    c1 = wave_sum_i(c1);
    m1 = wave_min_i(m1);
    c2 = wave_sum_i(c2);
    m2 = wave_min_i(m2);
    if ((threadIdx.x & 63) == 0) {
        s_cnt[0][threadIdx.x >> 6] = c1;
        s_min[0][threadIdx.x >> 6] = m1;
        s_cnt[1][threadIdx.x >> 6] = c2;
        s_min[1][threadIdx.x >> 6] = m2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int l = threadIdx.x;
        int c = 0, m = kIntMax;
        for (int i = 0; i < kBlock / 64; ++i) {
            c += s_cnt[l][i];
            m = m < s_min[l][i] ? m : s_min[l][i];
        }
        pc_next[l * kDiaPartMax + blockIdx.x] = c;
        pm_next[l * kDiaPartMax + blockIdx.x] = m;
    }
}

#define MPCG_DIA_CASES(X)                                                                                           \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

void launch_dia_round(hipStream_t s, const BfsBufs &b)
{
    int g = (b.nwords + kBlock - 1) / kBlock;   // one word per thread
    if (g > b.dia_grid) g = b.dia_grid;
    if (g > kDiaPartMax) g = kDiaPartMax;
    if (g < 1) g = 1;
    const int two = b.dia_two;   // two levels per launch
    const size_t lds2 = sizeof(uint32_t) * (2 * kBlock + 6 * (size_t)b.dia_R);
    for (int j = 0; j < kDiaRound; ++j) {
        const uint32_t *fc = (j & 1) ? b.df1 : b.df0;
        uint32_t *fn = (j & 1) ? b.df0 : b.df1;
        // per-block partials by launch parity (two levels each for the two-level kernel)
        const int32_t *pcc = b.part_cnt + (j & 1) * 2 * kDiaPartMax, *pmc = b.part_min + (j & 1) * 2 * kDiaPartMax;
        int32_t *pcn = b.part_cnt + ((j + 1) & 1) * 2 * kDiaPartMax;
        int32_t *pmn = b.part_min + ((j + 1) & 1) * 2 * kDiaPartMax;
        if (two) {
            switch (b.doff.nd) {
#define X(N)                                                                                                        \
    case N:                                                                                                         \
        hipLaunchKernelGGL(k_dia_level2<N>, dim3(g), dim3(kBlock), lds2, s, fc, fn, b.dv, b.dm, b.dist, b.nwords, \
                           j, b.dia_R, b.doff, pcc, pmc, pcn, pmn, b.st);                                           \
        break;
                X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
            default: break;
            }
            continue;
        }
        switch (b.doff.nd) {
#define X(N)                                                                                                        \
    case N:                                                                                                         \
        hipLaunchKernelGGL(k_dia_level<N>, dim3(g), dim3(kBlock), 0, s, fc, fn, b.dv, b.dm, b.dist, b.nwords, j,    \
                           b.doff, pcc, pmc, pcn, pmn, b.st);                                                       \
        break;
            MPCG_DIA_CASES(X)
#undef X
        default: break;
        }
    }
    hipLaunchKernelGGL(k_dia_round_end, dim3(1), dim3(64), 0, s, b.st, (two ? 2 : 1) * kDiaRound);
}

// ------------------------------- several levels per launch: temporal tiles --
//
// A block owns the words [a, e) of a tile and loads the frontier of level L0
// over [a - hR, e + hR) (R: the most words a diagonal's window reaches, so a
// level's words need the previous level's within R of them).  It then forms
// h levels in LDS, each over a range R words narrower on both sides than the
// last, so after h levels its own words are exact; the halo work is redone by
// the neighbouring blocks.  Frontier and visited bits of the range live in
// LDS, the masks of a thread's words in registers (patterns with at most
// kDiaTileDiags diagonals).  Each level's count and smallest new vertex (own words only) go
// to a ring of kDiaRing slots indexed by level; block 0 retires the previous
// launch's levels at the start (first empty level: finish) and clears the
// slots of the next launch's levels.  The distances, the stop, the
// eccentricity and the farthest vertex are the per-level kernels' integers.


template <int ND>
__global__ void __launch_bounds__(kDiaTileThreads)
k_dia_multi(const uint32_t *__restrict__ fin, uint32_t *__restrict__ fout, uint32_t *dv,
            const uint32_t *__restrict__ dm, int32_t *dist, int32_t nw, int32_t L0, int32_t h, int32_t T, int32_t R,
            DiaOffs o, int32_t *ring_cnt, int32_t *ring_min, DevState *st)
{
    // F: frontier bits of the loaded range at LDS index kDiaPad + (w - lo),
    // zero outside it, so that a window needs no bounds test (words outside
    // [0, nw) fall in the zero parts; R <= kDiaPad)
    constexpr int kF = kDiaTileWords + 2 * kDiaPad;
    __shared__ uint32_t F[2][kF];
    __shared__ uint32_t V[kDiaTileWords];
    __shared__ int s_cnt[kDiaMaxLevels], s_min[kDiaMaxLevels];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < 64) {
        // Wave 0 of block 0 retires the previous launch's levels (level 0 at
        // the first launch), lane l taking level first + l, all loads at once.
        const int done = st->bfs_done;
        const int first = L0 - h + 1 < 0 ? 0 : L0 - h + 1;
        const int nl = L0 - first + 1;
        const int lam = first + tid;
        int c = 1, mprev = kIntMax;
        if (tid < nl) {
            c = ring_cnt[lam % kDiaRing];
            if (lam > 0) mprev = ring_min[(lam - 1) % kDiaRing];
        }
        const unsigned long long zero = __ballot(tid < nl && c == 0);
        const int z = zero ? __ffsll((long long)zero) - 1 : nl;   // first empty level's lane
        const int vis = wave_sum_i(tid < z ? c : 0);
        if (!done) {
            if (tid == 0) st->bfs_visited += vis;
            if (zero && tid == z) {
                st->bfs_ecc = lam - 1;
                st->bfs_far = mprev;
                st->bfs_done = 1;
            }
            if (tid < h) {   // the slots of the next launch's levels
                ring_cnt[(L0 + h + 1 + tid) % kDiaRing] = 0;
                ring_min[(L0 + h + 1 + tid) % kDiaRing] = kIntMax;
            }
        }
    }
    if (tid < kDiaMaxLevels) {
        s_cnt[tid] = 0;
        s_min[tid] = kIntMax;
    }
    const int a = blockIdx.x * T;
    const int e = a + T < nw ? a + T : nw;
    const int lo = a - h * R > 0 ? a - h * R : 0;
    const int hi = e + h * R < nw ? e + h * R : nw;
    for (int i = tid; i < kF; i += kDiaTileThreads) {
        if (i < kDiaPad || i >= kDiaPad + (hi - lo)) F[0][i] = 0u;
        F[1][i] = 0u;
    }
    // thread-owned words w = lo + tid + j kDiaTileThreads; their masks stay in
    // registers for the launch (all loads issued together)
    uint32_t mr[kDiaPerThread][ND];
#pragma unroll
    for (int j = 0; j < kDiaPerThread; ++j) {
        const int w = lo + tid + j * kDiaTileThreads;
        const int wc = w < hi ? w : hi - 1;
#pragma unroll
        for (int t = 0; t < ND; ++t) mr[j][t] = dm[(size_t)t * nw + wc];
        if (w < hi) {
            F[0][kDiaPad + w - lo] = fin[w];
            V[w - lo] = dv[w];
        }
    }
    __syncthreads();
    for (int l = 0; l < h; ++l) {
        const uint32_t *cur = F[l & 1];
        uint32_t *nxt = F[(l + 1) & 1];
        const int shrink = (h - l - 1) * R;
        const int vl = a - shrink > lo ? a - shrink : lo;
        const int vh = e + shrink < hi ? e + shrink : hi;
        int cnt = 0, mn = kIntMax;
#pragma unroll
        for (int j = 0; j < kDiaPerThread; ++j) {
            int w = lo + tid + j * kDiaTileThreads;
            // opaque per level: the window indices derived from w are formed
            // here, not hoisted out of the level loop (96 live registers)
            asm volatile("" : "+v"(w));
            if (w >= vl && w < vh) {
                const int iw = kDiaPad + w - lo;
                uint32_t nb = 0u;
#pragma unroll
                for (int t = 0; t < ND; ++t) {
                    const int i0 = iw + o.q[t];
                    uint32_t win = cur[i0];
                    if (o.r[t]) win = __builtin_amdgcn_alignbit(cur[i0 + 1], win, o.r[t]);
                    nb |= win & mr[j][t];
                }
                const uint32_t vis = V[w - lo];
                nb &= ~vis;
                nxt[iw] = nb;
                if (nb) {
                    V[w - lo] = vis | nb;
                    if (w >= a && w < e) {
                        cnt += __popc(nb);
                        const int v0 = 32 * w + __ffs(nb) - 1;
                        mn = mn < v0 ? mn : v0;
                        for (uint32_t bb = nb; bb; bb &= bb - 1u) dist[32 * w + __ffs(bb) - 1] = L0 + l + 1;
                    }
                }
            }
        }
        cnt = wave_sum_i(cnt);
        mn = wave_min_i(mn);
        if ((tid & 63) == 0 && cnt) {
            atomicAdd(&s_cnt[l], cnt);
            atomicMin(&s_min[l], mn);
        }
        __syncthreads();
    }
    const uint32_t *fl = F[h & 1];
    for (int w = a + tid; w < e; w += kDiaTileThreads) {   // changed words only: see k_dia_clear
        const uint32_t fw = fl[kDiaPad + w - lo], vw = V[w - lo];
        if (fw) fout[w] = fw;
        if (vw != dv[w]) dv[w] = vw;   // only this block writes its own words
    }
    if (tid < h && s_cnt[tid]) {
        atomicAdd(&ring_cnt[(L0 + tid + 1) % kDiaRing], s_cnt[tid]);
        atomicMin(&ring_min[(L0 + tid + 1) % kDiaRing], s_min[tid]);
    }
}

__global__ void k_dia_ring_seed(int32_t *ring_cnt, int32_t *ring_min, int32_t src)
{
    const int t = threadIdx.x;
    if (t < kDiaRing) {
        ring_cnt[t] = t == 0 ? 1 : 0;
        ring_min[t] = t == 0 ? src : kIntMax;
    }
}

void launch_dia_ring_seed(hipStream_t s, const BfsBufs &b, int32_t src)
{
    hipLaunchKernelGGL(k_dia_ring_seed, dim3(1), dim3(kDiaRing), 0, s, b.ring_cnt, b.ring_min, src);
}

int launch_dia_multi_round(hipStream_t s, const BfsBufs &b, int launches, int k)
{
    const int g = (b.nwords + b.dia_T - 1) / b.dia_T;
    for (int l = 0; l < launches; ++l, ++k) {
        const uint32_t *fin = (k & 1) ? b.df1 : b.df0;
        uint32_t *fout = (k & 1) ? b.df0 : b.df1;
        switch (b.doff.nd) {
#define X(N)                                                                                                        \
    case N:                                                                                                         \
        hipLaunchKernelGGL(k_dia_multi<N>, dim3(g), dim3(kDiaTileThreads), 0, s, fin, fout, b.dv, b.dm, b.dist,     \
                           b.nwords, k * b.dia_h, b.dia_h, b.dia_T, b.dia_R, b.doff, b.ring_cnt, b.ring_min, b.st); \
        break;
            X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
        default: break;
        }
    }
    return k;
}

}  // namespace mpcg
