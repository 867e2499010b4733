/*
 * mpcg_oracle.c -- plain, slow CPU oracle for the restarted mixed-precision
 * CG method (Prolubnikov, "Parameter Optimization for Restarted
 * Mixed-Precision Iterative Sparse Solver", arXiv 2412.08059).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the bench do.  It shares no code, header or table with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction: every
 * fused multiply-add below is an explicit fma()/fmaf() call).
 *
 * What each function follows:
 *   or_spmv64 / or_spmv32  -- the sparse product A d of the CG iteration
 *                             (section "Conjugate Gradient Method"); each row
 *                             is one multiply-add per stored entry (eq. 16),
 *                             here as an fma chain in CSR order from 0.
 *   or_bfs / or_pseudo_diameter -- the 2BFS procedure (section "Computing
 *                             Pseudo-Diameter of the Graph Matrix") and its
 *                             per-component maximum for disconnected graphs.
 *   or_jacobi_solve        -- Algorithm I with the Jacobi method in place
 *                             of CG (section on rounding-error growth in other
 *                             iterative methods; the paper's Jacobi table).
 *   or_diameter_multi      -- 2BFS repeated from several starts (the remark
 *                             after the procedure) and the effective diameter
 *                             of Remark 1 from the starts' distances.
 *   or_knn_select          -- weighted kNN (section "Finding the Optimal
 *                             Tolerance ... via a Classification Approach":
 *                             min-max normalisation, squared Euclidean search,
 *                             1/rho weights of eq. (23)).
 *   or_solve               -- Algorithm I (explicit eps1), Algorithm II
 *                             (eps1 = AUTO: k0 FP32 iterations, v of eq. (13),
 *                             kNN, continue), and FP64-only CG (eps1 = NONE);
 *                             with precond = 1 every CG stage is the "CG with
 *                             preconditioning" procedure (subsection
 *                             "Propagation of Rounding Errors When Precondition
 *                             is Applied") with the Jacobi preconditioner
 *                             M = diag(A) that the subsection names.
 *
 * Readings where the paper is silent (all documented in the design notes):
 *   - tolerance is relative to ||b||_2 unless tol_mode = 1 (absolute);
 *   - the loop test uses the recursive residual sqrt(gamma); the true
 *     residual b - Ax is formed at the restart and at the final check;
 *   - FP32-phase dot products accumulate in FP64 (each FP32 x FP32 product is
 *     exact in FP64); alpha and beta are rounded to FP32;
 *   - 2BFS starts at the smallest vertex of each component; farthest-vertex
 *     ties go to the smallest index; self-loops are ignored;
 *   - kNN: loop from sample k+1 with strict '<'; the evicted member is the
 *     farthest one (ties: largest sample index); zero-distance neighbours
 *     vote by count; class-score ties go to the larger eps1 (smaller t).
 *   - preconditioned CG: the listing's start r_0 <- M^-1 (b - A x_0), d_0 <- r_0
 *     is read as r_0 = b - A x_0, d_0 = M^-1 r_0 (its loop then is the standard
 *     recurrence: alpha = r.M^-1 r / d.A d, beta = r'.M^-1 r' / r.M^-1 r,
 *     d' = M^-1 r' + beta d); z = M^-1 r is r_i / a_ii, one division per
 *     element in the working precision; the stop test is on ||r|| as in the
 *     unpreconditioned stages; a missing or non-positive diagonal entry (no
 *     SPD matrix has one) is reported as not SPD.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Row loops (the products and the element-wise vector updates) may run on
 * several host threads: each iteration writes only its own element, so the
 * result is the same bits as one thread.  Dot products and the BFS stay
 * sequential.  or_set_threads(1) (the default) runs everything on one thread. */
static int g_threads = 1;
#define OR_ROWS _Pragma("omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)")

void or_set_threads(int32_t t) { g_threads = t > 1 ? t : 1; }
int32_t or_get_threads(void) { return g_threads; }

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOTSPD (-2)
#define OR_ENOCONV (-3)
#define OR_ENOMEM (-4)
#define OR_ENONFINITE (-6)
#define OR_ENOMODEL (-9)

#define OR_FLAG_FP32_BREAKDOWN 1
#define OR_FLAG_FP32_MAXIT 2
#define OR_FLAG_FINAL_RESTARTED 4
#define OR_FLAG_KNN_EXACT 8

typedef struct {
    int32_t k0;           /* FP32 iterations used for v (Algorithm II) */
    int32_t tol_mode;     /* 0: relative to ||b||, 1: absolute */
    int32_t max_restarts; /* extra FP64 restarts after a failed final check */
    int32_t knn_k;        /* 0: take k from the model */
    int32_t precond;      /* 0: none, 1: Jacobi (M = diag(A)) */
    int32_t dot_acc;      /* FP32-phase dot products: 0 accumulate in FP64, 1 in FP32 */
    int64_t maxit1;       /* FP32 iteration cap, <=0: n */
    int64_t maxit2;       /* FP64 iteration cap, <=0: max(10n, 1000) */
} or_opts;

typedef struct {
    int64_t ns;            /* training samples */
    const double *feat;    /* ns x 4 raw features (n, m, ell, v) */
    const int32_t *label;  /* class t in 2..7 */
    const double *fmin;    /* 4 */
    const double *fmax;    /* 4 */
    int32_t k;
    int32_t mask;          /* bit j set: feature j used */
} or_model;

typedef struct {
    int32_t status, n1, n2, restarts, flags, k0_used, eps1_class, pad;
    double eps1_used, v, beta_b, relres_sp, relres_restart_true, relres_final_true;
    int64_t ell, bfs_t, bfs_u, ncomp;
} or_stats;

/* ---------------------------------------------------------------- SpMV -- */

void or_spmv64(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
               const double *x, double *y)
{
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            acc = fma(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

void or_spmv32(int64_t n, const int64_t *rp, const int32_t *col, const float *val,
               const float *x, float *y)
{
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            acc = fmaf(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

/* ----------------------------------------------------------------- BFS -- */

/* Breadth-first search from src over the stored pattern (self-loops ignored).
 * dist[] must be n long; unreached vertices get -1.  Returns the eccentricity
 * of src (largest finite distance). */
int32_t or_bfs(int64_t n, const int64_t *rp, const int32_t *col, int64_t src, int32_t *dist)
{
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t head = 0, tail = 0;
    int32_t ecc = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int64_t u = queue[head++];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
            int64_t v = col[k];
            if (v == u || dist[v] >= 0) continue;
            dist[v] = dist[u] + 1;
            if (dist[v] > ecc) ecc = dist[v];
            queue[tail++] = v;
        }
    }
    free(queue);
    return ecc;
}

/* BFS restricted to the vertices reachable from src, using caller scratch.
 * Returns the number of reached vertices; *far gets the farthest vertex
 * (ties: smallest index) and *ecc its distance.  dist entries of reached
 * vertices are reset to -1 before returning. */
static int64_t bfs_component(const int64_t *rp, const int32_t *col, int64_t src,
                             int32_t *dist, int64_t *queue, unsigned char *visited,
                             int64_t *far, int32_t *ecc)
{
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    if (visited) visited[src] = 1;
    while (head < tail) {
        int64_t u = queue[head++];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
            int64_t v = col[k];
            if (v == u || dist[v] >= 0) continue;
            dist[v] = dist[u] + 1;
            queue[tail++] = v;
            if (visited) visited[v] = 1;
        }
    }
    int64_t best = src;
    int32_t bd = 0;
    for (int64_t q = 0; q < tail; ++q) {
        int64_t v = queue[q];
        if (dist[v] > bd || (dist[v] == bd && v < best)) { bd = dist[v]; best = v; }
    }
    for (int64_t q = 0; q < tail; ++q) dist[queue[q]] = -1;
    *far = best;
    *ecc = bd;
    return tail;
}

/* 2BFS pseudo-diameter, taken per connected component and maximised.
 * out[0] = ell, out[1] = t, out[2] = u of the first component (in order of
 * its smallest vertex) attaining the maximum, out[3] = number of components. */
int or_pseudo_diameter(int64_t n, const int64_t *rp, const int32_t *col, int64_t *out)
{
    if (n <= 0) return OR_EINVAL;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *visited = (unsigned char *)calloc((size_t)n, 1);
    if (!dist || !queue || !visited) { free(dist); free(queue); free(visited); return OR_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t ell = -1, bt = 0, bu = 0, ncomp = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (visited[s]) continue;
        ++ncomp;
        int64_t t, u;
        int32_t e1, e2;
        bfs_component(rp, col, s, dist, queue, visited, &t, &e1);
        bfs_component(rp, col, t, dist, queue, NULL, &u, &e2);
        if (e2 > ell) { ell = e2; bt = t; bu = u; }
    }
    out[0] = ell; out[1] = bt; out[2] = bu; out[3] = ncomp;
    free(dist); free(queue); free(visited);
    return OR_OK;
}

/* ------------------------------------------------------ Jacobi method -- */

/* Algorithm I with the Jacobi method in place of CG (the section on the
 * matrix graph diameter and rounding-error growth in other iterative
 * methods): x_{k+1} = D^{-1}(b - (L + U) x_k), A = L + D + U.  One iteration
 * in the working precision: s_i = sum over the stored off-diagonal entries of
 * row i of a_ij x_j (fma chain in CSR order from 0), t_i = b_i - s_i, the
 * residual of the iterate r_i = t_i - a_ii x_i (one fma) and
 * x_{k+1,i} = t_i / a_ii.  ||r_k||^2 is summed in FP64 in row order; the
 * stage stops with x_k when ||r_k|| <= thr, when it is not finite, or when k
 * reaches the stage's iteration cap.  Returns the stop reason (1 converged,
 * 2 cap, 4 non-finite) and the number of updates in *iters. */
static int jac32_stage(int64_t n, const int64_t *rp, const int32_t *col, const float *v32, const float *d32,
                       const float *b32, float *x, float *xn, double thr, int64_t maxit, int64_t *iters,
                       double *g_out, float **ans)
{
    float *cur = x, *nxt = xn;
    for (int64_t k = 0;; ++k) {
        double g = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            float s = 0.0f;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
                if (col[e] != i) s = fmaf(v32[e], cur[col[e]], s);
            const float t = b32[i] - s;
            const float r = fmaf(-d32[i], cur[i], t);
            nxt[i] = t / d32[i];
            g = fma((double)r, (double)r, g);
        }
        *g_out = g;
        *iters = k;
        *ans = cur;
        if (!isfinite(g)) return 4;
        if (sqrt(g) <= thr) return 1;
        if (k >= maxit) return 2;
        float *tmp = cur; cur = nxt; nxt = tmp;
    }
}

static int jac64_stage(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *d,
                       const double *b, double *x, double *xn, double thr, int64_t maxit, int64_t *iters,
                       double *g_out, double **ans)
{
    double *cur = x, *nxt = xn;
    for (int64_t k = 0;; ++k) {
        double g = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
                if (col[e] != i) s = fma(val[e], cur[col[e]], s);
            const double t = b[i] - s;
            const double r = fma(-d[i], cur[i], t);
            nxt[i] = t / d[i];
            g = fma(r, r, g);
        }
        *g_out = g;
        *iters = k;
        *ans = cur;
        if (!isfinite(g)) return 4;
        if (sqrt(g) <= thr) return 1;
        if (k >= maxit) return 2;
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
}

/* eps1 = -1: FP64 stage only.  x gets the FP64 stage's answer. */
int or_jacobi_solve(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *b,
                    double *x, double eps1, double eps2, const or_opts *opts, or_stats *st)
{
    memset(st, 0, sizeof(*st));
    st->eps1_class = -1;
    if (n <= 0 || !(eps2 > 0.0) || (eps1 != -1.0 && !(eps1 > 0.0))) return st->status = OR_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(b[i])) return st->status = OR_ENONFINITE;
    for (int64_t e = 0; e < rp[n]; ++e)
        if (!isfinite(val[e])) return st->status = OR_ENONFINITE;
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *xa = (double *)malloc(sizeof(double) * (size_t)n);
    double *xb = (double *)malloc(sizeof(double) * (size_t)n);
    float *d32 = (float *)malloc(sizeof(float) * (size_t)n);
    float *b32 = (float *)malloc(sizeof(float) * (size_t)n);
    float *v32 = (float *)malloc(sizeof(float) * (size_t)(rp[n] > 0 ? rp[n] : 1));
    float *ya = (float *)malloc(sizeof(float) * (size_t)n);
    float *yb = (float *)malloc(sizeof(float) * (size_t)n);
    int rc = OR_OK;
    if (!d || !xa || !xb || !d32 || !b32 || !v32 || !ya || !yb) { rc = OR_ENOMEM; goto done; }
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] == i) d[i] = val[e];
        if (!(d[i] > 0.0)) { rc = OR_ENOTSPD; goto done; }
        d32[i] = (float)d[i];
        b32[i] = (float)b[i];
    }
    for (int64_t e = 0; e < rp[n]; ++e) v32[e] = (float)val[e];
    double bb = 0.0;
    for (int64_t i = 0; i < n; ++i) bb = fma(b[i], b[i], bb);
    const double bn = sqrt(bb);
    const int abs_tol = opts && opts->tol_mode == 1;
    const int64_t maxit1 = opts && opts->maxit1 > 0 ? opts->maxit1 : n;
    const int64_t maxit2 = opts && opts->maxit2 > 0 ? opts->maxit2 : (10 * n > 1000 ? 10 * n : 1000);
    int64_t it = 0;
    double g = 0.0;
    if (eps1 != -1.0) {
        for (int64_t i = 0; i < n; ++i) ya[i] = 0.0f;
        float *ans32 = ya;
        const int why = jac32_stage(n, rp, col, v32, d32, b32, ya, yb, abs_tol ? eps1 : eps1 * bn, maxit1, &it,
                                    &g, &ans32);
        st->n1 = (int32_t)it;
        if (why == 2) st->flags |= OR_FLAG_FP32_MAXIT;
        if (why == 4) st->flags |= OR_FLAG_FP32_BREAKDOWN;
        st->relres_sp = bn > 0.0 ? sqrt(g) / bn : 0.0;
        for (int64_t i = 0; i < n; ++i) xa[i] = (double)ans32[i];
        st->eps1_used = eps1;
    } else {
        for (int64_t i = 0; i < n; ++i) xa[i] = 0.0;
        st->eps1_used = -1.0;
    }
    double *ans = xa;
    const int why = jac64_stage(n, rp, col, val, d, b, xa, xb, abs_tol ? eps2 : eps2 * bn, maxit2, &it, &g, &ans);
    st->n2 = (int32_t)it;
    st->relres_final_true = bn > 0.0 ? sqrt(g) / bn : 0.0;
    memcpy(x, ans, sizeof(double) * (size_t)n);
    rc = why == 1 ? OR_OK : (why == 4 ? OR_ENONFINITE : OR_ENOCONV);
done:
    free(d); free(xa); free(xb); free(d32); free(b32); free(v32); free(ya); free(yb);
    return st->status = rc;
}

/* Multi-start 2BFS and an effective-diameter estimate (the remark after the
 * 2BFS procedure: repeat 2BFS from several start vertices and keep the
 * largest pseudo-diameter; Remark 1: the effective diameter is the distance
 * within which a share q of the vertex pairs lie).  For every start s: a BFS
 * from s gives t_s (farthest, smallest index on ties) and the distances from
 * s, which are tallied; a BFS from t_s gives l(t_s, u_s).  The effective
 * diameter is the smallest d >= 1 with (tally of distances 1..d) >= q * (all
 * tallied pairs), compared in double.
 * out[0] = standard pseudo-diameter, out[1] = max over it and the starts'
 * 2BFS values, out[2] = effective diameter (0 without pairs), out[3] =
 * number of pairs, out[4] = index of the first start that raised the
 * maximum (-1 if none). */
int or_diameter_multi(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *starts,
                      int32_t count, double q, int64_t *out)
{
    if (n <= 0 || count < 0 || !(q > 0.0 && q <= 1.0)) return OR_EINVAL;
    for (int32_t i = 0; i < count; ++i)
        if (starts[i] < 0 || starts[i] >= n) return OR_EINVAL;
    int64_t std4[4];
    int st = or_pseudo_diameter(n, rp, col, std4);
    if (st != OR_OK) return st;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *tally = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!dist || !tally) { free(dist); free(tally); return OR_ENOMEM; }
    int64_t best = std4[0], best_i = -1;
    for (int32_t i = 0; i < count; ++i) {
        or_bfs(n, rp, col, starts[i], dist);
        int64_t t = starts[i];
        int32_t td = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (dist[v] >= 1) tally[dist[v]] += 1;
            if (dist[v] > td || (dist[v] == td && v < t && dist[v] >= 0)) { td = dist[v]; t = v; }
        }
        int32_t e2 = or_bfs(n, rp, col, t, dist);
        if (e2 > best) { best = e2; best_i = i; }
    }
    int64_t pairs = 0, eff = 0, cum = 0;
    for (int64_t d = 1; d < n; ++d) pairs += tally[d];
    for (int64_t d = 1; d < n && pairs > 0; ++d) {
        cum += tally[d];
        if ((double)cum >= q * (double)pairs) { eff = d; break; }
    }
    out[0] = std4[0]; out[1] = best; out[2] = eff; out[3] = pairs; out[4] = best_i;
    free(dist); free(tally);
    return OR_OK;
}

/* ----------------------------------------------------------------- kNN -- */

static double knn_norm(double x, double lo, double hi)
{
    if (hi == lo) return 0.0;
    return (x - lo) / (hi - lo);
}

/* Weighted kNN over raw training features.  scores[t-2] receives the class
 * scores for t = 2..7.  Returns the class t (2..7) or a negative status. */
int or_knn_select(const or_model *m, const double *query, int32_t k_override,
                  double *scores, int32_t *exact)
{
    if (!m || m->ns <= 0) return OR_ENOMODEL;
    int64_t ns = m->ns;
    int32_t k = k_override > 0 ? k_override : m->k;
    if (k <= 0) return OR_EINVAL;
    if (k > ns) k = (int32_t)ns;
    double q[4];
    for (int j = 0; j < 4; ++j) q[j] = knn_norm(query[j], m->fmin[j], m->fmax[j]);
    double *d2 = (double *)malloc(sizeof(double) * (size_t)ns);
    int64_t *set = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    for (int64_t i = 0; i < ns; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) {
            if (!(m->mask & (1 << j))) continue;
            double s = knn_norm(m->feat[i * 4 + j], m->fmin[j], m->fmax[j]);
            double diff = q[j] - s;
            double sq = diff * diff;
            acc = acc + sq;
        }
        d2[i] = acc;
    }
    for (int32_t a = 0; a < k; ++a) set[a] = a;
    for (int64_t i = k; i < ns; ++i) {
        int32_t far = 0;
        for (int32_t a = 1; a < k; ++a) {
            int64_t ca = set[a], cf = set[far];
            if (d2[ca] > d2[cf] || (d2[ca] == d2[cf] && ca > cf)) far = a;
        }
        if (d2[i] < d2[set[far]]) set[far] = i;
    }
    /* ascending sample order for the weighted sums */
    for (int32_t a = 1; a < k; ++a) {
        int64_t key = set[a];
        int32_t b = a - 1;
        while (b >= 0 && set[b] > key) { set[b + 1] = set[b]; --b; }
        set[b + 1] = key;
    }
    double sc[6] = {0, 0, 0, 0, 0, 0};
    int zero = 0;
    for (int32_t a = 0; a < k; ++a) if (d2[set[a]] == 0.0) zero = 1;
    for (int32_t a = 0; a < k; ++a) {
        int64_t i = set[a];
        int32_t t = m->label[i];
        if (t < 2 || t > 7) { free(d2); free(set); return OR_EINVAL; }
        if (zero) {
            if (d2[i] == 0.0) sc[t - 2] = sc[t - 2] + 1.0;
        } else {
            sc[t - 2] = sc[t - 2] + 1.0 / sqrt(d2[i]);
        }
    }
    int32_t best = 2;
    for (int32_t t = 3; t <= 7; ++t)
        if (sc[t - 2] > sc[best - 2]) best = t;
    if (scores) for (int j = 0; j < 6; ++j) scores[j] = sc[j];
    if (exact) *exact = zero;
    free(d2); free(set);
    return best;
}

/* ------------------------------------------------------------------ CG -- */

static double dot64(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = fma(a[i], b[i], s);
    return s;
}

/* Dot product of two FP32 vectors.  acc32 = 0: the products are summed in
 * FP64 (each FP32 x FP32 product is exact in FP64); acc32 = 1: the whole sum
 * is an FP32 fma chain, returned widened. */
static double dot32(int64_t n, const float *a, const float *b, int acc32)
{
    if (acc32) {
        float s = 0.0f;
        for (int64_t i = 0; i < n; ++i) s = fmaf(a[i], b[i], s);
        return (double)s;
    }
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = fma((double)a[i], (double)b[i], s);
    return s;
}

/* r = b - A x (FP64), returns ||r||^2 */
static double true_residual(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                            const double *b, const double *x, double *r)
{
    or_spmv64(n, rp, col, val, x, r);
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    return dot64(n, r, r);
}

static int all_finite(int64_t n, const double *a)
{
    for (int64_t i = 0; i < n; ++i) if (!isfinite(a[i])) return 0;
    return 1;
}

static const double k_eps_class[8] = {0, 0, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7};

typedef struct {
    int64_t n;
    const int64_t *rp; const int32_t *col;
    const float *val;
    const float *dg;      /* diagonal of A~ (Jacobi), or NULL: no preconditioner */
    float *x, *r, *d, *q, *z;
    int acc32;            /* dot products accumulated in FP32 (dot_acc = 1) */
    double gamma;         /* r.r (stop test, v ratios) */
    double rho;           /* r.M^-1 r (alpha, beta); equals gamma without a preconditioner */
} cg32_state;

/* z = M^-1 r and rho = r.z for the current residual. */
static void precond32(cg32_state *s)
{
    if (s->dg) {
        float *z = s->z;
        const float *r = s->r, *dg = s->dg;
        OR_ROWS
        for (int64_t i = 0; i < s->n; ++i) z[i] = r[i] / dg[i];
        s->rho = dot32(s->n, s->r, s->z, s->acc32);
    } else {
        s->rho = s->gamma;
    }
}

/* One FP32 CG iteration.  Returns 0 on success, 1 on breakdown (delta not
 * positive or not finite; the iterate is left unchanged). */
static int cg32_step(cg32_state *s)
{
    int64_t n = s->n;
    float *x = s->x, *r = s->r, *d = s->d;
    const float *q = s->q;
    or_spmv32(n, s->rp, s->col, s->val, s->d, s->q);
    double delta = dot32(n, s->d, s->q, s->acc32);
    if (!isfinite(delta) || !(delta > 0.0)) return 1;
    float alpha = (float)(s->rho / delta);
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) {
        x[i] = fmaf(alpha, d[i], x[i]);
        r[i] = fmaf(-alpha, q[i], r[i]);
    }
    double rho_old = s->rho;
    s->gamma = dot32(n, s->r, s->r, s->acc32);
    precond32(s);
    float beta = (float)(s->rho / rho_old);
    const float *src = s->dg ? s->z : s->r;   /* M^-1 r' */
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) d[i] = fmaf(beta, d[i], src[i]);
    return 0;
}

/* Diagonal of A (the entry with col == row); 0 if a row has none. */
static void diagonal(int64_t n, const int64_t *rp, const int32_t *col, const double *val, double *dg)
{
    for (int64_t i = 0; i < n; ++i) {
        dg[i] = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] == i) dg[i] = val[k];
    }
}

/* FP64 CG state of the second stage: residual r = b - A x, direction d and
 * (Jacobi) z = M^-1 r; gamma = r.r, rho = r.z (= gamma without a
 * preconditioner). */
static void start64(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *dg64,
                    const double *b, const double *x, double *r, double *d, double *z, double *gamma,
                    double *rho)
{
    *gamma = true_residual(n, rp, col, val, b, x, r);
    *rho = *gamma;
    if (dg64) {
        OR_ROWS
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / dg64[i];
        *rho = dot64(n, r, z);
    }
    const double *src = dg64 ? z : r;
    OR_ROWS
    for (int64_t i = 0; i < n; ++i) d[i] = src[i];
}

/* Algorithm I / II and FP64-only CG.  x0 (may be NULL: zero) is the initial
 * guess of the first stage that runs: float32(x0) for the FP32 stage, x0
 * itself for FP64-only CG. */
int or_solve(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
             const double *b, const double *x0, double *x, double eps1, double eps2,
             const or_opts *opt_in, const or_model *model, or_stats *st)
{
    or_opts opt = {20, 0, 5, 0, 0, 0, 0, 0};
    if (opt_in) opt = *opt_in;
    or_stats S;
    memset(&S, 0, sizeof(S));
    S.eps1_class = -1;
    S.ell = -1;
    int status = OR_OK;
    if (n <= 0 || !rp || !b || !x || !(eps2 > 0.0) || !isfinite(eps2) ||
        !(eps1 == 0.0 || eps1 == -1.0 || (eps1 > 0.0 && isfinite(eps1)))) {
        if (st) { S.status = OR_EINVAL; *st = S; }
        return OR_EINVAL;
    }
    int64_t nnz = rp[n];
    if (rp[0] != 0) status = OR_EINVAL;
    for (int64_t i = 0; i < n && status == OR_OK; ++i) {
        if (rp[i + 1] < rp[i]) { status = OR_EINVAL; break; }
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n) { status = OR_EINVAL; break; }
            if (k > rp[i] && col[k] <= col[k - 1]) { status = OR_EINVAL; break; }
        }
    }
    if (status != OR_OK) { if (st) { S.status = status; *st = S; } return status; }
    if (!all_finite(nnz, val) || !all_finite(n, b) || (x0 && !all_finite(n, x0))) {
        if (st) { S.status = OR_ENONFINITE; *st = S; }
        return OR_ENONFINITE;
    }
    if (eps1 == 0.0 && (!model || model->ns <= 0)) {
        if (st) { S.status = OR_ENOMODEL; *st = S; }
        return OR_ENOMODEL;
    }
    if (opt.precond < 0 || opt.precond > 1 || opt.dot_acc < 0 || opt.dot_acc > 1) {
        if (st) { S.status = OR_EINVAL; *st = S; }
        return OR_EINVAL;
    }
    double *dg64 = NULL;
    if (opt.precond == 1) {
        dg64 = (double *)malloc(sizeof(double) * (size_t)n);
        diagonal(n, rp, col, val, dg64);
        for (int64_t i = 0; i < n; ++i) {
            if (!(dg64[i] > 0.0)) {
                free(dg64);
                if (st) { S.status = OR_ENOTSPD; *st = S; }
                return OR_ENOTSPD;
            }
        }
    }
    int64_t maxit1 = opt.maxit1 > 0 ? opt.maxit1 : n;
    int64_t maxit2 = opt.maxit2 > 0 ? opt.maxit2 : (10 * n > 1000 ? 10 * n : 1000);

    double beta_b = sqrt(dot64(n, b, b));
    S.beta_b = beta_b;
    if (beta_b == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        free(dg64);
        if (st) { S.status = OR_OK; *st = S; }
        return OR_OK;
    }
    double scale = opt.tol_mode == 1 ? 1.0 : beta_b;

    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);

    if (eps1 != -1.0) {
        /* ---- first stage: FP32 copy of A and b, x~ = float32(x0) ---- */
        float *val32 = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
        cg32_state s;
        float *dg32 = NULL;
        s.n = n; s.rp = rp; s.col = col; s.val = val32;
        s.acc32 = opt.dot_acc;
        s.x = (float *)malloc(sizeof(float) * (size_t)n);
        s.r = (float *)malloc(sizeof(float) * (size_t)n);
        s.d = (float *)malloc(sizeof(float) * (size_t)n);
        s.q = (float *)malloc(sizeof(float) * (size_t)n);
        s.z = (float *)malloc(sizeof(float) * (size_t)n);
        for (int64_t k = 0; k < nnz; ++k) val32[k] = (float)val[k];
        if (dg64) {   /* the diagonal of A~ */
            dg32 = (float *)malloc(sizeof(float) * (size_t)n);
            for (int64_t i = 0; i < n; ++i) dg32[i] = (float)dg64[i];
        }
        s.dg = dg32;
        if (x0) {
            /* r~ = b~ - A~ x~0, the product in FP32 */
            for (int64_t i = 0; i < n; ++i) s.x[i] = (float)x0[i];
            or_spmv32(n, rp, col, val32, s.x, s.q);
            for (int64_t i = 0; i < n; ++i) s.r[i] = (float)b[i] - s.q[i];
        } else {
            for (int64_t i = 0; i < n; ++i) {
                s.x[i] = 0.0f;
                s.r[i] = (float)b[i];      /* r~ = b~ - A~ * 0 */
            }
        }
        s.gamma = dot32(n, s.r, s.r, s.acc32);
        precond32(&s);
        for (int64_t i = 0; i < n; ++i) s.d[i] = dg32 ? s.z[i] : s.r[i];   /* d_0 = M^-1 r_0 */
        int64_t n1 = 0;
        int broke = 0;
        double e1 = eps1;
        if (eps1 == 0.0) {
            /* Algorithm II: k0 iterations, v = mean ||r_i|| / ||r_{i-1}|| */
            double sum = 0.0;
            int32_t used = 0;
            while (used < opt.k0 && s.gamma > 0.0) {
                double gprev = s.gamma;
                if (cg32_step(&s)) { broke = 1; break; }
                ++n1;
                double ratio = sqrt(s.gamma) / sqrt(gprev);
                sum = sum + ratio;
                ++used;
            }
            S.k0_used = used;
            S.v = used > 0 ? sum / (double)used : 0.0;
            int64_t pd[4];
            or_pseudo_diameter(n, rp, col, pd);
            S.ell = pd[0]; S.bfs_t = pd[1]; S.bfs_u = pd[2]; S.ncomp = pd[3];
            double chi[4] = {(double)n, (double)nnz, (double)pd[0], S.v};
            int32_t ex = 0;
            int cls = or_knn_select(model, chi, opt.knn_k, NULL, &ex);
            if (cls < 0) {
                status = cls;
                free(val32); free(s.x); free(s.r); free(s.d); free(s.q); free(s.z); free(dg32);
                goto done;
            }
            S.eps1_class = cls;
            if (ex) S.flags |= OR_FLAG_KNN_EXACT;
            e1 = k_eps_class[cls];
        }
        S.eps1_used = e1;
        if (broke) {
            S.flags |= OR_FLAG_FP32_BREAKDOWN;
        } else {
            for (;;) {
                if (sqrt(s.gamma) <= e1 * scale) break;
                if (n1 >= maxit1) { S.flags |= OR_FLAG_FP32_MAXIT; break; }
                if (cg32_step(&s)) { S.flags |= OR_FLAG_FP32_BREAKDOWN; break; }
                ++n1;
            }
        }
        S.n1 = (int32_t)n1;
        S.relres_sp = sqrt(s.gamma) / beta_b;
        for (int64_t i = 0; i < n; ++i) x[i] = (double)s.x[i];   /* float64(x~) */
        free(val32); free(s.x); free(s.r); free(s.d); free(s.q); free(s.z); free(dg32);
    } else {
        S.eps1_used = -1.0;
        for (int64_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    }

    /* ---- second stage: FP64 CG from x0 = float64(x~) with a true residual ---- */
    {
        double thr = eps2 * scale;
        double gamma, rho;
        start64(n, rp, col, val, dg64, b, x, r, d, z, &gamma, &rho);
        S.relres_restart_true = sqrt(gamma) / beta_b;
        int64_t n2 = 0;
        int32_t restarts = 0;
        for (;;) {
            while (!(sqrt(gamma) <= thr)) {
                if (n2 >= maxit2) { status = OR_ENOCONV; goto final; }
                or_spmv64(n, rp, col, val, d, q);
                double delta = dot64(n, d, q);
                if (!isfinite(delta)) { status = OR_ENONFINITE; goto final; }
                if (!(delta > 0.0)) { status = OR_ENOTSPD; goto final; }
                double alpha = rho / delta;
                OR_ROWS
                for (int64_t i = 0; i < n; ++i) {
                    x[i] = fma(alpha, d[i], x[i]);
                    r[i] = fma(-alpha, q[i], r[i]);
                }
                gamma = dot64(n, r, r);
                double rho_new = gamma;
                if (dg64) {
                    OR_ROWS
                    for (int64_t i = 0; i < n; ++i) z[i] = r[i] / dg64[i];
                    rho_new = dot64(n, r, z);
                }
                double beta = rho_new / rho;
                const double *src = dg64 ? z : r;
                OR_ROWS
                for (int64_t i = 0; i < n; ++i) d[i] = fma(beta, d[i], src[i]);
                rho = rho_new;
                ++n2;
            }
            /* final check on the true residual; if it fails, CG starts again
             * from x with r = b - A x (gamma and rho of that residual) */
            double res_true = sqrt(true_residual(n, rp, col, val, b, x, q));
            S.relres_final_true = res_true / beta_b;
            if (res_true <= thr) break;
            if (restarts >= opt.max_restarts) { status = OR_ENOCONV; break; }
            ++restarts;
            S.flags |= OR_FLAG_FINAL_RESTARTED;
            start64(n, rp, col, val, dg64, b, x, r, d, z, &gamma, &rho);
        }
    final:
        S.n2 = (int32_t)n2;
        S.restarts = restarts;
        if (status != OR_OK && S.relres_final_true == 0.0) {
            double res_true = sqrt(true_residual(n, rp, col, val, b, x, q));
            S.relres_final_true = res_true / beta_b;
        }
    }
done:
    free(r); free(d); free(q); free(z); free(dg64);
    S.status = status;
    if (st) *st = S;
    return status;
}

/* ------------------------------------------------- diagnostics for pins -- */

/* First nd search directions of FP64 CG from x0 = 0 (row-major nd x n).
 * Returns the number of directions recorded (fewer if CG stopped exactly). */
int64_t or_cg64_directions(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                           const double *b, int64_t nd, double *dirs)
{
    double *x = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i]; d[i] = b[i]; }
    double gamma = dot64(n, r, r);
    int64_t got = 0;
    for (; got < nd; ++got) {
        memcpy(dirs + got * n, d, sizeof(double) * (size_t)n);
        if (gamma == 0.0) { ++got; break; }
        or_spmv64(n, rp, col, val, d, q);
        double delta = dot64(n, d, q);
        if (!(delta > 0.0)) { ++got; break; }
        double alpha = gamma / delta;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = fma(alpha, d[i], x[i]);
            r[i] = fma(-alpha, q[i], r[i]);
        }
        double gnew = dot64(n, r, r);
        double beta = gnew / gamma;
        for (int64_t i = 0; i < n; ++i) d[i] = fma(beta, d[i], r[i]);
        gamma = gnew;
    }
    free(x); free(r); free(d); free(q);
    return got;
}

/* Plain CG from x0 = 0 entirely in one precision (prec = 32 or 64) for
 * `iters` iterations; true_res[i] = ||b - A x_i|| in FP64 for i = 0..iters. */
void or_cg_true_residuals(int32_t prec, int64_t n, const int64_t *rp, const int32_t *col,
                          const double *val, const double *b, int64_t iters, double *true_res)
{
    int64_t nnz = rp[n];
    double *xd = (double *)calloc((size_t)n, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (prec == 32) {
        float *val32 = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
        cg32_state s;
        s.n = n; s.rp = rp; s.col = col; s.val = val32;
        s.dg = NULL;
        s.z = NULL;
        s.acc32 = 0;
        s.x = (float *)calloc((size_t)n, sizeof(float));
        s.r = (float *)malloc(sizeof(float) * (size_t)n);
        s.d = (float *)malloc(sizeof(float) * (size_t)n);
        s.q = (float *)malloc(sizeof(float) * (size_t)n);
        for (int64_t k = 0; k < nnz; ++k) val32[k] = (float)val[k];
        for (int64_t i = 0; i < n; ++i) { s.r[i] = (float)b[i]; s.d[i] = s.r[i]; }
        s.gamma = dot32(n, s.r, s.r, 0);
        s.rho = s.gamma;
        for (int64_t it = 0; it <= iters; ++it) {
            for (int64_t i = 0; i < n; ++i) xd[i] = (double)s.x[i];
            true_res[it] = sqrt(true_residual(n, rp, col, val, b, xd, tmp));
            if (it == iters) break;
            if (s.gamma == 0.0 || cg32_step(&s)) {
                for (int64_t j = it + 1; j <= iters; ++j) true_res[j] = true_res[it];
                break;
            }
        }
        free(val32); free(s.x); free(s.r); free(s.d); free(s.q);
    } else {
        double *r = (double *)malloc(sizeof(double) * (size_t)n);
        double *d = (double *)malloc(sizeof(double) * (size_t)n);
        double *q = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) { r[i] = b[i]; d[i] = b[i]; }
        double gamma = dot64(n, r, r);
        for (int64_t it = 0; it <= iters; ++it) {
            true_res[it] = sqrt(true_residual(n, rp, col, val, b, xd, tmp));
            if (it == iters) break;
            or_spmv64(n, rp, col, val, d, q);
            double delta = dot64(n, d, q);
            if (gamma == 0.0 || !(delta > 0.0)) {
                for (int64_t j = it + 1; j <= iters; ++j) true_res[j] = true_res[it];
                break;
            }
            double alpha = gamma / delta;
            for (int64_t i = 0; i < n; ++i) {
                xd[i] = fma(alpha, d[i], xd[i]);
                r[i] = fma(-alpha, q[i], r[i]);
            }
            double gnew = dot64(n, r, r);
            double beta = gnew / gamma;
            for (int64_t i = 0; i < n; ++i) d[i] = fma(beta, d[i], r[i]);
            gamma = gnew;
        }
        free(r); free(d); free(q);
    }
    free(xd); free(tmp);
}

/* Coefficients of plain FP64 CG from x0 = 0 (no preconditioner), for the
 * CG-Lanczos estimate of the extreme eigenvalues of A: CG's step lengths
 * alpha_j and ratios beta_j = gamma_{j+1} / gamma_j define the tridiagonal
 * Lanczos matrix T_k with diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1} and
 * off-diagonal sqrt(beta_j)/alpha_j (Saad, "Iterative Methods for Sparse
 * Linear Systems", the CG-Lanczos connection), whose extreme eigenvalues
 * approach those of A.  Runs until ||r|| <= eps ||b|| or maxit iterations;
 * returns the number k of (alpha, beta) pairs written.  x_out (may be NULL)
 * gets the final iterate: the arithmetic is that of FP64-only CG in or_solve
 * up to its stop, before any final check. */
int64_t or_cg_lanczos(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                      const double *b, double eps, int64_t maxit, double *alpha_out, double *beta_out,
                      double *x_out)
{
    double *x = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i]; d[i] = b[i]; }
    double gamma = dot64(n, r, r);
    const double thr = eps * sqrt(gamma);
    int64_t k = 0;
    while (k < maxit && gamma > 0.0 && !(sqrt(gamma) <= thr)) {
        or_spmv64(n, rp, col, val, d, q);
        double delta = dot64(n, d, q);
        if (!(delta > 0.0)) break;
        double alpha = gamma / delta;
        OR_ROWS
        for (int64_t i = 0; i < n; ++i) {
            x[i] = fma(alpha, d[i], x[i]);
            r[i] = fma(-alpha, q[i], r[i]);
        }
        double gnew = dot64(n, r, r);
        double beta = gnew / gamma;
        OR_ROWS
        for (int64_t i = 0; i < n; ++i) d[i] = fma(beta, d[i], r[i]);
        alpha_out[k] = alpha;
        beta_out[k] = beta;
        gamma = gnew;
        ++k;
    }
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)n);
    free(x); free(r); free(d); free(q);
    return k;
}
