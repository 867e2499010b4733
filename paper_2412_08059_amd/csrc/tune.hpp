// Tuning table: the scheduling parameters of the products and the 2BFS per
// class of matrix and GPU (plain C++, no HIP).  Every parameter leaves the
// results unchanged -- it picks how loads are issued or how many blocks run a
// level, never what is summed in which order -- so a table written on one
// machine can only make another slower, not wrong.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mpcg.h"

namespace mpcg {

// A matrix class: the GPU (architecture name and compute units), whether the
// SELL-64 copy stores 16-bit column offsets, the mean row length and the row
// count, both on a log2 scale.
struct TuneKey {
    std::string arch;
    int32_t cu = 0, idx16 = 0, lenlog = 0, nlog = 0;
};

struct TuneEntry {
    TuneKey key;
    mpcg_tuning t{};
};

struct TuneTable {
    std::vector<TuneEntry> solve;   // per matrix class: the single-solve fields
    bool has_batch = false;         // the batch engine's fields, per GPU
    std::string batch_arch;
    int32_t batch_cu = 0;
    mpcg_tuning batch{};
};

mpcg_tuning tune_defaults();
bool tune_valid(const mpcg_tuning &t);
int32_t tune_lenlog(int64_t n, int64_t nnz);   // round(log2(max(1, nnz / n)))
int32_t tune_nlog(int64_t n);                  // floor(log2(n))
// 0, or MPCG_EINVAL for an unreadable or malformed file (the table is then unchanged).
int tune_load(const char *path, TuneTable *out);
// The solve fields for a matrix: among the entries of the same GPU, index
// width and row-length bucket, the one nearest in log2(n) (ties: the smaller
// n); the defaults if there is none.  band = largest |i - j| of the pattern.
mpcg_tuning tune_lookup(const TuneTable &tb, const std::string &arch, int32_t cu, int64_t n, int64_t nnz,
                        int64_t band);
// The batch engine's fields for this GPU, or the defaults.
mpcg_tuning tune_batch(const TuneTable &tb, const std::string &arch, int32_t cu);

}  // namespace mpcg
