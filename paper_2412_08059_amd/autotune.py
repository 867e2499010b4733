"""Autotuner of the library's scheduling parameters (mpcg_tuning).

    python -m paper_2412_08059_amd.autotune [--out PATH] [--quick]

On the GPU it runs, for representative matrices of each class (grids,
bands, random graphs at several sizes), every candidate of the parameters
that choose how a product issues its loads and how the 2BFS expands its
levels, times the kernels through the library (mpcg_time_kernel, mpcg_bfs,
Algorithm II solves), keeps the fastest candidate per class, then times a
mixed batch under candidate engine schedules, and writes the table that
Solver and BatchSolver load by default (tuning.txt beside this file).  The
parameters change no result (tests/test_gpu_tune.py checks every candidate
bit for bit), so the table only decides speed.

A matrix's class is the key of tune.cpp: the GPU (architecture name and
compute units), 16- or 32-bit SELL column offsets (largest |i - j| below
2^15 or not), round(log2(nnz / n)) and floor(log2(n)); a lookup takes the
nearest log2(n) among the entries that match the rest.
"""

from __future__ import annotations

import argparse
import math
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.txt")

SOLVE_FIELDS = ("sell_batch", "sell_whole_batch", "sell_split", "bfs_grid", "bfs_grid_shared", "bfs_persist",
                "bfs_dia", "bfs_dia_tiles", "sell_stream")
# the fields a table row may leave out, with their defaults (the C library's)
OPTIONAL_DEFAULTS = {"bfs_dia": 1, "bfs_dia_tiles": 1, "sell_stream": -1}
BATCH_FIELDS = ("batch_group_steps", "batch_bfs_rounds", "batch_small_cap", "batch_small_levels",
                "batch_level_grid", "batch_runahead", "batch_bfs_band")
BATCH_OPTIONAL_DEFAULTS = {"batch_runahead": 0, "batch_bfs_band": 1}


# ----------------------------------------------------------- class keys --

def lenlog(n: int, nnz: int) -> int:
    """round(log2(max(1, nnz / n))), halves away from zero (C's lround)."""
    mean = nnz / n if n > 0 else 1.0
    return int(math.floor(math.log2(max(1.0, mean)) + 0.5))


def nlog(n: int) -> int:
    return max(0, int(n).bit_length() - 1)


def band_of(a) -> int:
    import numpy as np
    rows = np.repeat(np.arange(a.n, dtype=np.int64), np.diff(a.row_ptr))
    return int(np.abs(a.col.astype(np.int64) - rows).max()) if a.nnz else 0


def class_key(arch: str, cu: int, a) -> tuple:
    return (arch, int(cu), 1 if band_of(a) < 32768 else 0, lenlog(a.n, a.nnz), nlog(a.n))


# ------------------------------------------------------------ selection --

def sell_candidates(idx16: int):
    """(sell_batch, sell_whole_batch, sell_split) candidates; the split only
    matters where the columns are 32-bit (scattered gathers)."""
    splits = (-1,) if idx16 else (0, 1)
    return [(b, w, sp) for b in (4, 8) for w in (0, 1, 2, 3) for sp in splits]


def choose_min(timings: dict):
    """The candidate of least time (ties: the first listed)."""
    best = None
    for cand, t in timings.items():
        if best is None or t < timings[best]:
            best = cand
    return best


# --------------------------------------------------------------- table --

def format_table(solve_rows: dict, batch_row, comment: str = "") -> str:
    """solve_rows: {class key: {field: value}}; batch_row: (arch, cu, {field:
    value}) or None.  Returns the text tune.cpp parses."""
    out = ["mpcg-tune 1"]
    if comment:
        out += ["# " + ln for ln in comment.splitlines()]
    out.append("# solve arch cu idx16 lenlog nlog sell_batch sell_whole_batch sell_split bfs_grid "
               "bfs_grid_shared bfs_persist bfs_dia bfs_dia_tiles sell_stream")
    for key in sorted(solve_rows):
        v = solve_rows[key]
        arch, cu, idx16, ll, nl = key
        out.append(f"solve {arch} {cu} {idx16} {ll} {nl} " + " ".join(str(int(v[f])) for f in SOLVE_FIELDS))
    if batch_row is not None:
        arch, cu, v = batch_row
        out.append("# batch arch cu group_steps bfs_rounds small_cap small_levels level_grid runahead bfs_band")
        v = {**BATCH_OPTIONAL_DEFAULTS, **v}
        out.append(f"batch {arch} {cu} " + " ".join(str(int(v[f])) for f in BATCH_FIELDS))
    return "\n".join(out) + "\n"


def parse_table(text: str):
    """Inverse of format_table (for tests and reports)."""
    solve_rows, batch_row = {}, None
    lines = [ln.strip() for ln in text.splitlines() if ln.strip() and not ln.strip().startswith("#")]
    if not lines or lines[0] != "mpcg-tune 1":
        raise ValueError("not an mpcg-tune 1 table")
    for ln in lines[1:]:
        f = ln.split()
        if f[0] == "solve" and 12 <= len(f) <= 6 + len(SOLVE_FIELDS):
            key = (f[1], int(f[2]), int(f[3]), int(f[4]), int(f[5]))
            row = dict(OPTIONAL_DEFAULTS)
            row.update(zip(SOLVE_FIELDS, (int(v) for v in f[6:])))
            solve_rows[key] = row
        elif f[0] == "batch" and 8 <= len(f) <= 3 + len(BATCH_FIELDS):
            row = dict(BATCH_OPTIONAL_DEFAULTS)
            row.update(zip(BATCH_FIELDS, (int(v) for v in f[3:])))
            batch_row = (f[1], int(f[2]), row)
        else:
            raise ValueError(f"bad line: {ln}")
    return solve_rows, batch_row


# --------------------------------------------------------------- sweeps --

def _matrices(quick: bool):
    import workloads as W
    mats = [("poisson2d_256", lambda: W.poisson2d(256)), ("poisson2d_1024", lambda: W.poisson2d(1024)),
            ("varcoef3d_32", lambda: W.varcoef3d(32, seed=0)), ("varcoef3d_64", lambda: W.varcoef3d(64, seed=0)),
            ("varcoef3d_128", lambda: W.varcoef3d(128, seed=0)),
            ("banded_100k", lambda: W.banded(100_000, 8, seed=0)), ("banded_1M", lambda: W.banded(1_000_000, 8, seed=0)),
            ("banded_4M", lambda: W.banded(4_000_000, 8, seed=0)),
            ("er_100k", lambda: W.er_laplacian(100_000, 16, seed=0)),
            ("er_1M", lambda: W.er_laplacian(1_000_000, 16, seed=0))]
    if quick:
        mats = [m for m in mats if m[0] in ("varcoef3d_32", "banded_100k", "er_100k")]
    return mats


def _time_kernels(capi, ctx, desc, reps):
    t64 = capi.mpcg_time_kernel(ctx, desc, capi.MPCG_KERNEL_CG_SPMV_F64, reps)
    t32 = capi.mpcg_time_kernel(ctx, desc, capi.MPCG_KERNEL_CG_SPMV_F32, reps)
    return t32, t64


def tune_solve(quick: bool = False, log=print):
    """Per class: the SELL load form and split, the 2BFS grid and mode, and
    the 2BFS grid beside Algorithm II's FP32 phase."""
    import torch
    import workloads as W
    from paper_2412_08059_amd import DEFAULT_MODEL, DeviceCSR, Solver, capi
    rows = {}
    arch = cu = None
    for name, gen in _matrices(quick):
        a = gen()
        _, b = W.rhs(a, seed=0)
        sv = Solver(a.n, a.nnz, model=DEFAULT_MODEL, tuning=None)
        if arch is None:
            props = torch.cuda.get_device_properties(0)
            arch = props.gcnArchName.split(":")[0]
            cu = props.multi_processor_count
        key = class_key(arch, cu, a)
        A = DeviceCSR.from_host(a)
        B = torch.from_numpy(b).cuda()
        X = torch.empty(a.n, dtype=torch.float64, device="cuda")
        reps = 5 if quick else 15
        sell = {}
        for cand in sell_candidates(key[2]):
            capi.mpcg_set_tuning(sv.ctx, dict(zip(("sell_batch", "sell_whole_batch", "sell_split"), cand)))
            t32, t64 = _time_kernels(capi, sv.ctx, A.desc, reps)
            sell[cand] = t32 + t64
        best_sell = choose_min(sell)
        # nontemporal matrix loads stay with the size rule (-1): a class spans
        # sizes on both sides of the Infinity Cache
        base = dict(zip(("sell_batch", "sell_whole_batch", "sell_split"), best_sell), sell_stream=-1)
        bfs = {}
        for persist in (0, 1):
            for grid in (64, 128, 256):
                capi.mpcg_set_tuning(sv.ctx, dict(base, bfs_grid=grid, bfs_persist=persist))
                ts = []
                for _ in range(2 if quick else 3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, _, _, _ = sv.bfs(A, 0)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                bfs[(grid, persist)] = statistics.median(ts)
        g, persist = choose_min(bfs)
        base.update(bfs_grid=g, bfs_persist=persist)
        dia = {}   # the 2BFS on diagonals (where the pattern has at most 16), one launch or tiles per level
        for cand in ((0, 1), (1, 0), (1, 1)):
            capi.mpcg_set_tuning(sv.ctx, dict(base, bfs_dia=cand[0], bfs_dia_tiles=cand[1]))
            ts = []
            for _ in range(2 if quick else 3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sv.bfs(A, 0)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            dia[cand] = statistics.median(ts)
        d, dt = choose_min(dia)
        base.update(bfs_dia=d, bfs_dia_tiles=dt)
        shared = {}
        for gs in (32, 64, 128):
            capi.mpcg_set_tuning(sv.ctx, dict(base, bfs_grid_shared=gs))
            sv.solve(A, B, 0.0, 1e-10, x=X)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sv.solve(A, B, 0.0, 1e-10, x=X)
            torch.cuda.synchronize()
            shared[gs] = time.perf_counter() - t0
        base.update(bfs_grid_shared=choose_min(shared))
        sv.close()
        prev = rows.get(key)
        rows[key] = base
        log(f"# tune {name} key={key}: {base} (sell best {sell[best_sell] * 1e3:.1f} us of "
            f"{min(sell.values()) * 1e3:.1f}..{max(sell.values()) * 1e3:.1f}){' (replaces an earlier entry)' if prev else ''}")
        del A, B, X
        torch.cuda.empty_cache()
    return arch, cu, rows


def tune_batch(arch: str, cu: int, quick: bool = False, log=print):
    """The batch engine's schedule on a mixed batch (four families, n
    log-uniform in [1e3, 5e4]), Algorithm II and FP64-only."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_08059_amd import DEFAULT_MODEL, BatchSolver, DeviceCSR
    rng = np.random.default_rng(77)
    systems = []
    for i in range(24 if quick else 96):
        fam = W.FAMILIES[int(rng.integers(0, len(W.FAMILIES)))]
        n = int(np.exp(rng.uniform(np.log(1e3), np.log(5e4))))
        a = W.family_matrix(fam, n, seed=500 + i)
        _, b = W.rhs(a, seed=500 + i)
        systems.append((DeviceCSR.from_host(a), torch.from_numpy(b).cuda(),
                        torch.empty(a.n, dtype=torch.float64, device="cuda"), a))
    rows = sum(((s[3].n + 63) // 64) * 64 for s in systems)
    nnz = sum(s[3].nnz for s in systems)
    cands = [dict(batch_group_steps=gs, batch_level_grid=lg, batch_small_cap=sc)
             for gs in (4, 8, 16) for lg in (512, 1024) for sc in (256, 512)]
    if quick:
        cands = cands[:3]
    res = {}
    for c in cands:
        eng = BatchSolver(rows, 2 * nnz + 64 * rows, len(systems), model=DEFAULT_MODEL, tuning=c)
        tot = 0.0
        for e1 in (0.0, -1.0):
            for rep in range(2):
                t0 = time.perf_counter()
                ids = eng.submit([(A, B, X, e1, 1e-10) for (A, B, X, _) in systems])
                eng.wait_all(ids, timeout_s=600)
                if rep:
                    tot += time.perf_counter() - t0
        eng.close()
        res[tuple(sorted(c.items()))] = tot
        log(f"# tune batch {c}: {tot * 1e3:.1f} ms (auto + FP64-only)")
    best = dict(choose_min(res))
    out = {"batch_group_steps": 8, "batch_bfs_rounds": 4, "batch_small_cap": 512, "batch_small_levels": 64,
           "batch_level_grid": 1024, **BATCH_OPTIONAL_DEFAULTS}
    out.update(best)
    return arch, cu, out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="three small matrices, few candidates (a check run)")
    ap.add_argument("--no-batch", action="store_true")
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    arch, cu, rows = tune_solve(args.quick, log)
    batch_row = None if args.no_batch else tune_batch(arch, cu, args.quick, log)
    text = format_table(rows, batch_row, comment=f"written by paper_2412_08059_amd/autotune.py on {arch} "
                                                 f"({cu} CUs) in {time.perf_counter() - t0:.0f} s")
    with open(args.out, "w") as f:
        f.write(text)
    log(f"# wrote {args.out} ({len(rows)} classes)")
    print(text, end="")


if __name__ == "__main__":
    main()
