// Host-side kNN model and selector (plain C++, no HIP).
#pragma once

#include <cstdint>

#include "mpcg.h"

namespace mpcg {

struct KnnModel {
    int32_t k = 0, mask = 15;
    double omega = 1.0 / 3.0;
    int64_t ns = 0;
    double *feat = nullptr;    // ns x 4 raw features (n, m, pseudo-diameter, v)
    int32_t *label = nullptr;  // class t in 2..7
    double fmin[4] = {0, 0, 0, 0}, fmax[4] = {0, 0, 0, 0};
};

int knn_load(const char *path, KnnModel *m);   // 0, or MPCG_EINVAL on a malformed file
void knn_free(KnnModel *m);
// Returns the class t in 2..7 (or a negative mpcg_status); *exact = 1 when a
// training sample is at distance zero.
int knn_select(const KnnModel &m, const double chi[4], int32_t k_override, int32_t *exact);

}  // namespace mpcg
