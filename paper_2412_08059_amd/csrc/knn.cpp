// Host-side weighted kNN selector of eps1 (section "Finding the Optimal
// Tolerance ... via a Classification Approach"): per-feature min-max
// normalisation from the training sample, squared Euclidean distance for the
// neighbour search, 1/rho weights (eq. 23), class t -> eps1 = 10^-t.
//
// Compiled with -ffp-contract=off so that the distance and weight arithmetic
// is the plain sequence of IEEE operations written here.
//
// Tie rules: the neighbour set starts as the first k samples and a later
// sample replaces the current farthest member only if it is strictly closer
// (the farthest member is the one with the largest distance, the largest
// sample index on equal distances) -- which leaves the k smallest samples in
// the order (distance, index), the set this file selects directly; if any
// neighbour is at distance zero only the zero-distance neighbours vote, one
// vote each; equal class scores go to the smaller t (the larger eps1).

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "knn.hpp"

namespace mpcg {

namespace {

double norm01(double x, double lo, double hi)
{
    if (hi == lo) return 0.0;
    return (x - lo) / (hi - lo);
}

bool next_data_line(FILE *f, std::string &line)
{
    char buf[4096];
    while (std::fgets(buf, sizeof(buf), f)) {
        const char *p = buf;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == '\0') continue;
        line.assign(p);
        return true;
    }
    return false;
}

}  // namespace

void knn_free(KnnModel *m)
{
    std::free(m->feat);
    std::free(m->label);
    m->feat = nullptr;
    m->label = nullptr;
    m->ns = 0;
}

int knn_load(const char *path, KnnModel *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return MPCG_EINVAL;
    KnnModel m;
    std::string line;
    bool ok = next_data_line(f, line) && line.rfind("mpcg-knn-model 1", 0) == 0;
    int have = 0;
    while (ok && have != 0x3f && next_data_line(f, line)) {
        char key[32] = {0};
        if (std::sscanf(line.c_str(), "%31s", key) != 1) { ok = false; break; }
        const char *rest = line.c_str() + std::strlen(key);
        if (!std::strcmp(key, "k")) { ok = std::sscanf(rest, "%d", &m.k) == 1; have |= 1; }
        else if (!std::strcmp(key, "mask")) { ok = std::sscanf(rest, "%d", &m.mask) == 1; have |= 2; }
        else if (!std::strcmp(key, "omega")) { ok = std::sscanf(rest, "%lf", &m.omega) == 1; have |= 4; }
        else if (!std::strcmp(key, "ns")) { long long v; ok = std::sscanf(rest, "%lld", &v) == 1; m.ns = v; have |= 8; }
        else if (!std::strcmp(key, "fmin")) {
            ok = std::sscanf(rest, "%lf %lf %lf %lf", &m.fmin[0], &m.fmin[1], &m.fmin[2], &m.fmin[3]) == 4;
            have |= 16;
        } else if (!std::strcmp(key, "fmax")) {
            ok = std::sscanf(rest, "%lf %lf %lf %lf", &m.fmax[0], &m.fmax[1], &m.fmax[2], &m.fmax[3]) == 4;
            have |= 32;
        } else {
            ok = false;
        }
    }
    if (ok && (have != 0x3f || m.ns <= 0 || m.k <= 0 || m.mask < 0 || m.mask > 15)) ok = false;
    if (ok) {
        m.feat = static_cast<double *>(std::malloc(sizeof(double) * 4 * (size_t)m.ns));
        m.label = static_cast<int32_t *>(std::malloc(sizeof(int32_t) * (size_t)m.ns));
        ok = m.feat && m.label;
        for (int64_t i = 0; ok && i < m.ns; ++i) {
            int t = 0;
            ok = next_data_line(f, line) &&
                 std::sscanf(line.c_str(), "%lf %lf %lf %lf %d", &m.feat[4 * i], &m.feat[4 * i + 1],
                             &m.feat[4 * i + 2], &m.feat[4 * i + 3], &t) == 5 &&
                 t >= 2 && t <= 7;
            if (ok) m.label[i] = t;
        }
    }
    std::fclose(f);
    if (!ok) {
        knn_free(&m);
        return MPCG_EINVAL;
    }
    *out = m;
    return 0;
}

int knn_select(const KnnModel &m, const double chi[4], int32_t k_override, int32_t *exact)
{
    if (m.ns <= 0) return MPCG_ENOMODEL;
    int64_t k = k_override > 0 ? k_override : m.k;
    if (k <= 0) return MPCG_EINVAL;
    if (k > m.ns) k = m.ns;
    // squared distance of every training sample to the query in the
    // normalised space, features in index order, one rounding per operation
    auto scaled = [&](double x, int j) { return norm01(x, m.fmin[j], m.fmax[j]); };
    std::vector<std::pair<double, int64_t>> cand((size_t)m.ns);
    for (int64_t i = 0; i < m.ns; ++i) {
        double d2 = 0.0;
        for (int j = 0; j < 4; ++j) {
            if ((m.mask >> j) & 1) {
                const double e = scaled(chi[j], j) - scaled(m.feat[4 * i + j], j);
                const double e2 = e * e;
                d2 = d2 + e2;
            }
        }
        cand[(size_t)i] = {d2, i};
    }
    // The tie rules (start from the first k samples; a later one replaces the
    // farthest member -- largest distance, then largest index -- only when
    // strictly closer) keep exactly the k smallest samples under the total
    // order (distance, index): select those.
    std::partial_sort(cand.begin(), cand.begin() + k, cand.end());
    cand.resize((size_t)k);
    // votes are added in ascending sample index
    std::sort(cand.begin(), cand.end(),
              [](const std::pair<double, int64_t> &x, const std::pair<double, int64_t> &y) { return x.second < y.second; });
    const bool at_zero = std::any_of(cand.begin(), cand.end(), [](const std::pair<double, int64_t> &c) {
        return c.first == 0.0;
    });
    double vote[6] = {0, 0, 0, 0, 0, 0};
    for (const auto &c : cand) {
        const int cls = m.label[c.second];
        if (at_zero) {
            if (c.first == 0.0) vote[cls - 2] = vote[cls - 2] + 1.0;   // exact matches vote by count
        } else {
            vote[cls - 2] = vote[cls - 2] + 1.0 / std::sqrt(c.first);   // eq. 23: weight 1/rho
        }
    }
    // the largest score wins; on equal scores the smaller t (larger eps1)
    int best = 2;
    for (int cls = 3; cls <= 7; ++cls)
        if (vote[cls - 2] > vote[best - 2]) best = cls;
    if (exact) *exact = at_zero ? 1 : 0;
    return best;
}

}  // namespace mpcg
