// Tuning table: parser and lookup (see tune.hpp).
//
// File format (text, '#' starts a comment line):
//   mpcg-tune 1
//   solve <arch> <cu> <idx16> <lenlog> <nlog> <sell_batch> <sell_whole_batch> <sell_split> <bfs_grid>
//         <bfs_grid_shared> <bfs_persist> [<bfs_dia> [<bfs_dia_tiles> [<sell_stream>]]]
//   batch <arch> <cu> <group_steps> <bfs_rounds> <small_cap> <small_levels> <level_grid>
//         [<runahead> [<bfs_band>]]

#include "tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace mpcg {

mpcg_tuning tune_defaults()
{
    mpcg_tuning t{};
    t.sell_batch = 4;
    t.sell_whole_batch = 1;   // FP32 products load whole batches, FP64 ones guard each entry
    t.sell_split = -1;        // two launches for 32-bit columns (scattered gathers)
    t.bfs_grid = 128;
    t.bfs_grid_shared = 64;
    t.bfs_persist = 0;
    t.batch_group_steps = 8;
    t.batch_bfs_rounds = 4;
    t.batch_small_cap = 512;
    t.batch_small_levels = 64;
    t.batch_level_grid = 1024;
    t.bfs_dia = 1;
    t.bfs_dia_tiles = 1;
    t.sell_stream = -1;
    t.batch_runahead = 0;
    t.batch_bfs_band = 1;
    return t;
}

bool tune_valid(const mpcg_tuning &t)
{
    return (t.sell_batch == 4 || t.sell_batch == 8) && t.sell_whole_batch >= 0 && t.sell_whole_batch <= 3 &&
           t.sell_split >= -1 && t.sell_split <= 1 && t.bfs_grid >= 1 && t.bfs_grid <= 4096 &&
           t.bfs_grid_shared >= 1 && t.bfs_grid_shared <= 4096 && (t.bfs_persist == 0 || t.bfs_persist == 1) &&
           t.batch_group_steps >= 1 && t.batch_group_steps <= 64 && t.batch_bfs_rounds >= 1 &&
           t.batch_bfs_rounds <= 64 && t.batch_small_cap >= 1 && t.batch_small_cap <= 2048 &&
           t.batch_small_levels >= 1 && t.batch_small_levels <= 4096 && t.batch_level_grid >= 1 &&
           t.batch_level_grid <= 65536 && t.bfs_dia >= 0 && t.bfs_dia <= 2 &&
           (t.bfs_dia_tiles == 0 || t.bfs_dia_tiles == 1) && t.sell_stream >= -1 && t.sell_stream <= 1 &&
           (t.batch_runahead >= 0 && t.batch_runahead <= 2) && (t.batch_bfs_band == 0 || t.batch_bfs_band == 1);
}

int32_t tune_lenlog(int64_t n, int64_t nnz)
{
    const double mean = n > 0 ? (double)nnz / (double)n : 1.0;
    return (int32_t)std::lround(std::log2(mean > 1.0 ? mean : 1.0));
}

int32_t tune_nlog(int64_t n)
{
    int32_t k = 0;
    while (n > 1) {
        n >>= 1;
        ++k;
    }
    return k;
}

int tune_load(const char *path, TuneTable *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return MPCG_EINVAL;
    TuneTable tb;
    char line[1024];
    bool header = false, ok = true;
    while (ok && std::fgets(line, sizeof(line), f)) {
        const char *p = line;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == '\0') continue;
        if (!header) {
            header = std::strncmp(p, "mpcg-tune 1", 11) == 0;
            ok = header;
            continue;
        }
        char kind[16] = {0}, arch[64] = {0};
        if (std::sscanf(p, "%15s %63s", kind, arch) != 2) { ok = false; break; }
        if (!std::strcmp(kind, "solve")) {
            TuneEntry e;
            e.t = tune_defaults();
            const int got = std::sscanf(p, "%*s %*s %d %d %d %d %d %d %d %d %d %d %d %d %d", &e.key.cu,
                                        &e.key.idx16, &e.key.lenlog, &e.key.nlog, &e.t.sell_batch,
                                        &e.t.sell_whole_batch, &e.t.sell_split, &e.t.bfs_grid, &e.t.bfs_grid_shared,
                                        &e.t.bfs_persist, &e.t.bfs_dia, &e.t.bfs_dia_tiles, &e.t.sell_stream);
            e.key.arch = arch;
            ok = got >= 10 && got <= 13 && tune_valid(e.t);   // the last three fields may be absent (defaults)
            if (ok) tb.solve.push_back(e);
        } else if (!std::strcmp(kind, "batch")) {
            mpcg_tuning t = tune_defaults();
            int cu = 0;
            const int got = std::sscanf(p, "%*s %*s %d %d %d %d %d %d %d %d", &cu, &t.batch_group_steps,
                                        &t.batch_bfs_rounds, &t.batch_small_cap, &t.batch_small_levels,
                                        &t.batch_level_grid, &t.batch_runahead, &t.batch_bfs_band);
            ok = got >= 6 && got <= 8 && tune_valid(t);   // the last two fields may be absent (defaults)
            if (ok) {
                tb.has_batch = true;
                tb.batch_arch = arch;
                tb.batch_cu = cu;
                tb.batch = t;
            }
        } else {
            ok = false;
        }
    }
    std::fclose(f);
    if (!ok || !header) return MPCG_EINVAL;
    *out = tb;
    return 0;
}

mpcg_tuning tune_lookup(const TuneTable &tb, const std::string &arch, int32_t cu, int64_t n, int64_t nnz,
                        int64_t band)
{
    const int32_t idx16 = band < 32768 ? 1 : 0;
    const int32_t lenlog = tune_lenlog(n, nnz), nlog = tune_nlog(n);
    const TuneEntry *best = nullptr;
    int32_t best_d = 0;
    for (const TuneEntry &e : tb.solve) {
        if (e.key.arch != arch || e.key.cu != cu || e.key.idx16 != idx16 || e.key.lenlog != lenlog) continue;
        const int32_t d = std::abs(e.key.nlog - nlog);
        if (!best || d < best_d || (d == best_d && e.key.nlog < best->key.nlog)) {
            best = &e;
            best_d = d;
        }
    }
    mpcg_tuning t = tune_defaults();
    if (best) {
        t.sell_batch = best->t.sell_batch;
        t.sell_whole_batch = best->t.sell_whole_batch;
        t.sell_split = best->t.sell_split;
        t.bfs_grid = best->t.bfs_grid;
        t.bfs_grid_shared = best->t.bfs_grid_shared;
        t.bfs_persist = best->t.bfs_persist;
        t.bfs_dia = best->t.bfs_dia;
        t.bfs_dia_tiles = best->t.bfs_dia_tiles;
        t.sell_stream = best->t.sell_stream;
    }
    return t;
}

mpcg_tuning tune_batch(const TuneTable &tb, const std::string &arch, int32_t cu)
{
    if (tb.has_batch && tb.batch_arch == arch && tb.batch_cu == cu) return tb.batch;
    return tune_defaults();
}

}  // namespace mpcg
