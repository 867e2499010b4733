#!/usr/bin/env python3
"""Time-to-1e-10 of the restarted mixed-precision CG (Algorithm II: features +
kNN eps1 + FP32 CG + FP64 restart) against FP64-only CG on the same GPU.

Workload: 3D 7-point variable-coefficient diffusion on a 128^3 grid
(n = 2,097,152, m = 14,581,760), face coefficients 10^U(0,3), x* ~ U[-1,1]
(seed 0), b = A x*, x0 = 0, eps2 = 1e-10.  Inputs are resident in HBM before
the timed region.

One step = one Algorithm II solve (ingest, 2BFS, k0 = 20 FP32 iterations, kNN,
FP32 CG to eps1, FP64 restart, FP64 CG, final true-residual check) plus one
FP64-only solve of the same system.  `value` is the mean time-to-1e-10 of the
mixed solve in ms.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-1e-10 residual, mixed vs FP64-only CG; SpMV GB/s vs HBM peak"


def kernel_bytes(kind: str, n: int, m: int) -> float:
    """Algorithmic HBM bytes of one launch (each array touched once; the
    x-gather counted once per vector, i.e. perfect reuse)."""
    s = 8 if kind.endswith("64") else 4
    if kind.startswith("cg_spmv"):
        # val + col, row pointers, gathers of r and d_old, x read and written
        # (the previous iteration's x += alpha d), writes of d_new and q
        return (s + 4) * m + 4 * (n + 1) + 6 * s * n
    if kind.startswith("update"):
        # reads r, q; writes r
        return 3 * s * n
    # plain y = A x
    return (s + 4) * m + 4 * (n + 1) + 2 * s * n


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration), or None
    when the summary is for another workload or the kernel's source file has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_varcoef3d_128.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        k = rec["kernels"][kernel]
        if rec.get("workload") != workload:
            return None
        with open(os.path.join(ROOT, k["source"]), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != k["source_sha1"]:
                return None
        return float(k["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def sell_format_bytes(kind: str, a) -> float:
    """HBM bytes the library's SELL-64 copy makes a launch move: every padded
    entry's value and stored column (16-bit offsets when the band allows,
    else 32-bit), the row pointers the slices read their lengths from, the
    slice offsets, and the vectors as in kernel_bytes (perfect gather reuse).
    Padded entries: 64 x the longest row of each 64-row slice."""
    import numpy as np
    s = 8 if kind.endswith("64") else 4
    n = a.n
    lens = np.diff(a.row_ptr)
    pad = np.zeros(((n + 63) // 64) * 64, dtype=np.int64)
    pad[:n] = lens
    padded = int(pad.reshape(-1, 64).max(axis=1).sum()) * 64
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    band = int(np.abs(a.col.astype(np.int64) - rows).max()) if a.nnz else 0
    cw = 2 if band < 32768 else 4
    mat = (s + cw) * padded + 4 * (n + 1) + 8 * (n // 64 + 1)
    if kind.startswith("cg_spmv"):
        return mat + 6 * s * n
    if kind.startswith("update"):
        return 3 * s * n
    return mat + 2 * s * n


def _host_info():
    info = {"nproc": len(os.sched_getaffinity(0)), "cpu_model": None}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except (OSError, ValueError):
        pass
    return info


def cpu_baseline(a, b, model_path, x_mixed, x_dp, n1, n2, n_dp):
    """The oracle on the host's cores, two legs:
    - all cores (its row loops on every thread; the same bits as one thread):
      Algorithm II with the packaged model (2BFS, v, kNN, FP32 then FP64 CG),
      timed in full, and FP64-only CG, whose CG-Lanczos coefficients give
      kappa-hat; their solutions are the reference for the GPU's errors;
    - one thread on a bounded sample (the 2BFS plus 20- and 40-iteration runs
      in each precision), extrapolated with the GPU's iteration counts."""
    import numpy as np
    import oracle
    host = _host_info()
    threads = max(1, min(16, host["nproc"]))
    oracle.set_threads(threads)
    try:
        model = oracle.load_model(model_path)
        t0 = time.perf_counter()
        r = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-10, model=model)
        t_mixed = time.perf_counter() - t0
        t0 = time.perf_counter()
        kap, lmin, lmax, k_dp, x_or_dp = oracle.lanczos_kappa(a, b, 1e-10, want_x=True)
        t_dp = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))

    t0 = time.perf_counter()
    oracle.pseudo_diameter(a)
    t_feat = time.perf_counter() - t0

    def timed(**kw):
        t = time.perf_counter()
        oracle.solve(a, b, **kw)
        return time.perf_counter() - t

    k = 20
    t32a = timed(eps1=1e-30, eps2=1e300, maxit1=k)
    t32b = timed(eps1=1e-30, eps2=1e300, maxit1=2 * k)
    t64a = timed(eps1=-1.0, eps2=1e-300, maxit2=k, max_restarts=0)
    t64b = timed(eps1=-1.0, eps2=1e-300, maxit2=2 * k, max_restarts=0)
    it32 = (t32b - t32a) / k
    it64 = (t64b - t64a) / k
    one_ms = (t_feat + n1 * it32 + n2 * it64) * 1e3
    return {
        "value": round(t_mixed * 1e3, 1),
        "unit": "ms",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the whole workload: the oracle's Algorithm II solve (class {r.eps1_class}, N1={r.n1}, "
                   f"N2={r.n2}) with its row loops on {threads} threads; FP64-only CG (N_dp={k_dp}) "
                   f"{t_dp * 1e3:.0f} ms; one-thread leg: 2BFS ({t_feat * 1e3:.0f} ms) and {k}/{2 * k}-iteration "
                   f"runs ({it32 * 1e3:.1f} / {it64 * 1e3:.1f} ms per FP32 / FP64 iteration) extrapolated with "
                   f"the GPU's N1={n1}, N2={n2}"),
        "fp64_only_ms": round(t_dp * 1e3, 1),
        "one_thread_ms": round(one_ms, 1),
        "one_thread_fp64_only_ms": round(n_dp * it64 * 1e3, 1),
        "omega_cpu_one_thread": round(it32 / it64, 3),
        "nproc": host["nproc"],
        "cpu_model": host["cpu_model"],
        "oracle_counts": {"eps1_class": r.eps1_class, "n1": r.n1, "n2": r.n2, "n_dp": k_dp},
        "kappa_hat": round(kap, 1),
        "err_vs_oracle": {"mixed": rel(x_mixed, r.x), "fp64_only": rel(x_dp, x_or_dp)},
    }


def _mixed_systems(count, n_lo, n_hi, seed):
    """`count` systems, family uniform over the four workload families, n
    log-uniform in [n_lo, n_hi], x* ~ U[-1,1], b = A x* (seed + i each)."""
    import numpy as np
    import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        fam = W.FAMILIES[int(rng.integers(0, len(W.FAMILIES)))]
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        a = W.family_matrix(fam, n, seed=seed + i)
        _, b = W.rhs(a, seed=seed + i)
        out.append((fam, a, b))
    return out


def _iter_bytes(n, m, n1, n2):
    """Algorithmic bytes of n1 FP32 and n2 FP64 CG iterations (product + update)."""
    it = lambda s: kernel_bytes("cg_spmv" + ("64" if s == 8 else "32"), n, m) + kernel_bytes(
        "update" + ("64" if s == 8 else "32"), n, m)
    return n1 * it(4) + n2 * it(8)


def bench_c1(args):
    """The paper's own regime: 2D Poisson 64^2 (n = 4,096), eps1 = 1e-4 and
    Algorithm II against FP64-only CG on the GPU (mean of repeated solves).
    At this size a CG iteration is launch- and latency-bound in both
    precisions."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_08059_amd import DEFAULT_MODEL, DeviceCSR, Solver
    a = W.poisson2d(64)
    xs, b = W.rhs(a, seed=args.seed)
    sv = Solver(a.n, a.nnz, model=DEFAULT_MODEL)
    A, B = DeviceCSR.from_host(a), torch.from_numpy(b).cuda()
    X = torch.empty(a.n, dtype=torch.float64, device="cuda")
    out = {}
    for label, e1 in (("eps1_1e-4", 1e-4), ("auto", 0.0), ("fp64_only", -1.0)):
        for _ in range(3):
            sv.solve(A, B, e1, 1e-10, x=X)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            st, _, S = sv.solve(A, B, e1, 1e-10, x=X)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[label] = {"ms": round(ms, 3), "n1": S.n1, "n2": S.n2, "status": st, "eps1": S.eps1_used,
                      "err_vs_xstar": float(np.linalg.norm(X.cpu().numpy() - xs) / np.linalg.norm(xs))}
    sv.close()
    out["speedup_eps1_1e-4_vs_fp64_only"] = round(out["fp64_only"]["ms"] / out["eps1_1e-4"]["ms"], 3)
    out["speedup_auto_vs_fp64_only"] = round(out["fp64_only"]["ms"] / out["auto"]["ms"], 3)
    return out


def bench_large_band(args):
    """Bandwidth outside the 256 MB Infinity Cache: the CG kernels on a band of
    n = 4e6 rows (half-width 8, the C3a recipe), whose FP64 CG product moves
    about 1 GB per launch.  HIP events over back-to-back launches on the
    library stream (mpcg_time_kernel)."""
    import workloads as W
    from paper_2412_08059_amd import DeviceCSR, Solver, capi
    t = time.perf_counter()
    a = W.banded(args.large_n, 8, seed=args.seed)
    print(f"# large band n={a.n} nnz={a.nnz} (generated in {time.perf_counter() - t:.1f}s)", file=sys.stderr,
          flush=True)
    sv = Solver(a.n, a.nnz)
    A = DeviceCSR.from_host(a)
    out = {"n": a.n, "m": a.nnz}
    for k, kid in (("cg_spmv_f64", capi.MPCG_KERNEL_CG_SPMV_F64), ("cg_spmv_f32", capi.MPCG_KERNEL_CG_SPMV_F32),
                   ("update_f64", capi.MPCG_KERNEL_UPDATE_F64), ("update_f32", capi.MPCG_KERNEL_UPDATE_F32),
                   ("spmv_f64", capi.MPCG_KERNEL_SPMV_F64)):
        ms = capi.mpcg_time_kernel(sv.ctx, A.desc, kid, 20)
        byt = kernel_bytes(k, a.n, a.nnz)
        fbyt = sell_format_bytes(k, a)
        out[k] = {"us": round(ms * 1e3, 2), "bytes": int(byt), "GBs": round(byt / (ms * 1e-3) / 1e9, 1),
                  "frac": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3), "format_bytes": int(fbyt),
                  "frac_format": round(fbyt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    sv.close()
    return out


def bench_batch(args):
    """Many independent systems in one engine: Algorithm II (kNN eps1), a fixed
    eps1 = 1e-4 control and FP64-only CG, each submitted as one batch."""
    import numpy as np
    import torch
    from paper_2412_08059_amd import DEFAULT_MODEL, BatchSolver, DeviceCSR
    t = time.perf_counter()
    systems = _mixed_systems(args.batch_count, args.batch_nmin, args.batch_nmax, args.seed + 1000)
    rows = sum(((a.n + 63) // 64) * 64 for _, a, _ in systems)
    nnz = sum(a.nnz for _, a, _ in systems)
    print(f"# batch: {len(systems)} systems, {rows} padded rows, {nnz} nonzeros "
          f"(generated in {time.perf_counter() - t:.1f}s)", file=sys.stderr, flush=True)
    dev = [(DeviceCSR.from_host(a), torch.from_numpy(b).cuda(),
            torch.empty(a.n, dtype=torch.float64, device="cuda")) for _, a, b in systems]
    eng = BatchSolver(rows, 2 * nnz + 64 * rows, len(systems), model=DEFAULT_MODEL)
    res = {}
    for label, e1 in (("auto", 0.0), ("fixed_1e-4", 1e-4), ("fp64_only", -1.0)):
        for rep in range(1 + args.warmup):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids = eng.submit([(A, B, X, e1, 1e-10) for (A, B, X) in dev])
            got = eng.wait_all(ids, timeout_s=1800)
            wall = time.perf_counter() - t0
        st = [got[i][0] for i in ids]
        bad = [s.status for s in st if s.status != 0 or s.relres_final_true > 1e-10]
        n1 = [s.n1 for s in st]
        n2 = [s.n2 for s in st]
        byt = sum(_iter_bytes(a.n, a.nnz, s.n1, s.n2) for (_, a, _), s in zip(systems, st))
        res[label] = {"wall_ms": round(wall * 1e3, 1), "solves_per_s": round(len(st) / wall, 1),
                      "sum_n1": int(np.sum(n1)), "sum_n2": int(np.sum(n2)), "failed": len(bad),
                      "cg_GBs": round(byt / wall / 1e9, 1),
                      "latency_ms_p50": round(float(np.percentile([s.t_total_ms for s in st], 50)), 1),
                      "latency_ms_max": round(float(np.max([s.t_total_ms for s in st])), 1)}
        if e1 == 0.0:
            tf = [s.t_feat_ms for s in st]
            res[label]["features_ms_p50"] = round(float(np.percentile(tf, 50)), 1)
            res[label]["features_ms_p90"] = round(float(np.percentile(tf, 90)), 1)
            res[label]["eps1_classes"] = {str(t): int(sum(1 for s in st if s.eps1_class == t)) for t in range(2, 8)}
        print(f"# batch {label}: {res[label]}", file=sys.stderr, flush=True)
    eng.close()
    fams = {f: sum(1 for g, _, _ in systems if g == f) for f in ("lap2d", "lap3d", "banded", "er")}
    out = {"metric": "batched solves/s, 512 SPD systems, time-to-1e-10 each", "value": res["auto"]["solves_per_s"],
           "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": f"{len(systems)} systems, n log-uniform [{args.batch_nmin:g}, {args.batch_nmax:g}], "
                                  f"families {fams}, x*~U[-1,1], b=Ax*, eps2=1e-10",
                      "rows": rows, "nnz": nnz},
           "speedup_vs_fp64_only": round(res["fp64_only"]["wall_ms"] / res["auto"]["wall_ms"], 3),
           "modes": res}
    print(json.dumps(out))


def bench_family(args):
    """The paper's kNN experiment on its three matrix families (perturbed
    extended stars, random tree + floor(c n) edges, random bands of density p;
    Algorithm III values; mu in {1.1, 3, 10}) at n ~ 1000: GPU labelling of
    every matrix through the batch engine (features, N1/N2 for each eps1,
    FP64-only), then Acc, Loc, E and E_opt (eq. 27) over random
    training/test splits with the library's kNN."""
    import numpy as np
    from paper_2412_08059_amd import DEFAULT_MODEL, BatchSolver, Solver, family_eval as FE
    from workloads import paper_family as PF
    n = args.family_n
    sizes = {"star": n + 1, "random": n, "banded": n}
    eng = BatchSolver(256 * (n + 128), 256 * 200_000, 256, model=DEFAULT_MODEL, dot_acc=args.dot_acc)
    solver = None if args.family_no_omega else Solver(n + 8, 200_000, dot_acc=args.dot_acc)
    fams = {}
    for fam in ("star", "random", "banded"):
        specs = PF.sample_specs(fam, sizes[fam], scale=args.family_scale, seed=args.seed)
        t = time.perf_counter()
        mats = [PF.make(sp) for sp in specs]
        tgen = time.perf_counter() - t
        print(f"# family {fam} n={sizes[fam]}: {len(mats)} matrices (generated in {tgen:.1f}s)",
              file=sys.stderr, flush=True)
        rows, secs = FE.label(mats, lambda a, i: PF.paper_rhs(a, 7919 * i + 1)[1], eng, omega_solver=solver)
        print(f"# family {fam}: labelled in {secs:.1f}s ({8 * len(rows) / secs:.0f} solves/s)",
              file=sys.stderr, flush=True)
        res = FE.evaluate(rows, reps=args.family_reps, seed=args.seed)
        res["label_s"] = round(secs, 1)
        res["solves_per_s"] = round(8 * len(rows) / secs, 1)
        fams[fam] = res
        print(f"# family {fam}: {json.dumps(res)}", file=sys.stderr, flush=True)
    eng.close()
    if solver is not None:
        solver.close()
    e5 = [fams[f]["per_k"]["5"]["E_third"][0] for f in fams]
    out = {"metric": "paper-family kNN experiment: E (eq. 27, omega = 1/3, k = 5) mean over the three families",
           "value": round(float(np.mean(e5)), 2), "unit": "%", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": f"perturbed extended stars n={n + 1}, random tree + cn edges n={n}, random bands "
                                  f"n={n}; Algorithm III values; mu in {{1.1, 3, 10}}; x~U(1,2), b=Ax; eps2=1e-10; "
                                  f"sample scale {args.family_scale} of the appendix sizes; "
                                  f"{args.family_reps} training/test splits",
                      "features": "(m, pseudo-diameter, v)",
                      "fp32_dot_accumulation": "fp32" if args.dot_acc else "fp64"},
           "paper_context": {"Acc_pct_n1000": [70, 71, 74], "E_third_pct_n1000": [22, 22, 17.7],
                             "E_meas_pct_n1000": [31.0, 30.8, 25.3], "note": "sequential CPU, Colab"},
           "families": fams}
    print(json.dumps(out))


def bench_diameter(args):
    """Diameter contrast at n = 1M: a band of half-width 8 (pseudo-diameter
    ~n/8) and an Erdos-Renyi graph Laplacian of mean degree 16 (diameter ~5).
    For each: the feature pass, the kNN eps1, Algorithm I at every candidate
    eps1 and FP64-only CG; I = omega N1 + N2 at omega = 1/3 and at the
    measured omega, and the regret I(chosen) / I(best) - 1."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_08059_amd import DEFAULT_MODEL, DeviceCSR, Solver
    from paper_2412_08059_amd.model_builder import iteration_omega
    out_cases = {}
    for name, gen in (("banded_1M", lambda: W.banded(1_000_000, 8, seed=args.seed)),
                      ("er_1M", lambda: W.er_laplacian(1_000_000, 16, seed=args.seed))):
        a = gen()
        _, b = W.rhs(a, seed=args.seed)
        sv = Solver(a.n, a.nnz, model=DEFAULT_MODEL)
        A = DeviceCSR.from_host(a)
        B = torch.from_numpy(b).cuda()
        X = torch.empty(a.n, dtype=torch.float64, device="cuda")
        st, f = sv.features(A, B, 20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, f = sv.features(A, B, 20)
        torch.cuda.synchronize()
        t_feat = (time.perf_counter() - t0) * 1e3
        omega = iteration_omega(sv, A)

        def timed(e1):
            sv.solve(A, B, e1, 1e-10, x=X)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, _, S = sv.solve(A, B, e1, 1e-10, x=X)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3, st, S

        sweep = []
        for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
            ms, st, S = timed(e)
            sweep.append({"eps1": e, "ms": round(ms, 2), "n1": S.n1, "n2": S.n2, "status": st})
        ms_dp, st_dp, S_dp = timed(-1.0)
        ms_auto, st_auto, S_auto = timed(0.0)
        n1 = np.array([r["n1"] for r in sweep], float)
        n2 = np.array([r["n2"] for r in sweep], float)
        chosen = S_auto.eps1_class - 2
        res = {}
        for tag, w in (("third", 1.0 / 3.0), ("measured", omega)):
            I = w * n1 + n2
            best = int(np.argmin(I))
            res[tag] = {"omega": round(w, 4), "I_best": round(float(I[best]), 1), "eps1_best": sweep[best]["eps1"],
                        "I_chosen": round(float(I[chosen]), 1), "regret": round(float(I[chosen] / I[best] - 1.0), 4),
                        "I_dp": S_dp.n2}
        out_cases[name] = {"n": a.n, "m": a.nnz, "pdiam": f.pdiam, "v": round(f.v, 6), "n_components": f.n_components,
                           "t_feat_ms": round(t_feat, 2), "eps1_chosen": S_auto.eps1_used,
                           "auto_ms": round(ms_auto, 2), "auto_n1": S_auto.n1, "auto_n2": S_auto.n2,
                           "fp64_only_ms": round(ms_dp, 2), "speedup_vs_fp64_only": round(ms_dp / ms_auto, 3),
                           "sweep": sweep, "cost": res}
        print(f"# diameter {name}: {json.dumps(out_cases[name])}", file=sys.stderr, flush=True)
        sv.close()
    reg = [out_cases[c]["cost"]["third"]["regret"] for c in out_cases]
    out = {"metric": "diameter contrast: kNN eps1 regret I(chosen)/I(best) - 1 at omega = 1/3 (mean of the two)",
           "value": round(float(np.mean(reg)), 4), "unit": "ratio", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": "banded n=1M half-width 8 (a_ij ~ U[-1,0), a_ii = row |sum| + 1e-4) and "
                                  "Erdos-Renyi n=1M mean degree 16 (L = D - Adj + 1e-3 I); x*~U[-1,1], b=Ax*, "
                                  "eps2=1e-10"},
           "cases": out_cases}
    print(json.dumps(out))


def bench_jacobi_iter(args):
    """Algorithm I with the Jacobi method (two-stage Jacobi) against FP64-only
    Jacobi on a paper-family banded matrix (full bandwidth 17, density 0.8 --
    dense enough that no vertex is isolated, which Jacobi could not divide by
    -- Algorithm III values, mu = 3, so the Jacobi contraction factor is at
    most 1/3), n = 2^21."""
    import numpy as np
    import torch
    from paper_2412_08059_amd import DeviceCSR, Solver
    from workloads import paper_family as PF
    n = args.jac_n
    t = time.perf_counter()
    a = PF.random_banded(n, 17, 0.8, 3.0, seed=args.seed)
    _, b = PF.paper_rhs(a, args.seed)
    print(f"# jacobi_iter: n={a.n} nnz={a.nnz} (generated in {time.perf_counter() - t:.1f}s)", file=sys.stderr,
          flush=True)
    sv = Solver(a.n, a.nnz)
    A = DeviceCSR.from_host(a)
    B = torch.from_numpy(b).cuda()
    X = torch.empty(a.n, dtype=torch.float64, device="cuda")
    runs = {}
    for label, e1 in [("fp64_only", -1.0)] + [(f"eps1_{e:g}", e) for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]:
        ms = []
        for rep in range(1 + args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _, S = sv.solve_jacobi(A, B, e1, 1e-10, x=X)
            torch.cuda.synchronize()
            if rep > args.warmup:
                ms.append((time.perf_counter() - t0) * 1e3)
        runs[label] = {"ms": round(float(np.mean(ms)), 3), "n1": S.n1, "n2": S.n2, "status": st,
                       "relres_final_true": S.relres_final_true, "t_sp_ms": round(S.t_sp_ms, 3),
                       "t_dp_ms": round(S.t_dp_ms, 3)}
        print(f"# jacobi_iter {label}: {runs[label]}", file=sys.stderr, flush=True)
    from paper_2412_08059_amd import capi
    kus = {}
    for kname, kid in (("jacobi_f64", capi.MPCG_KERNEL_JACOBI_F64), ("jacobi_f32", capi.MPCG_KERNEL_JACOBI_F32)):
        kus[kname] = capi.mpcg_time_kernel(sv.ctx, A.desc, kid, 30) * 1e3
    sv.close()
    bad = {k: v["status"] for k, v in runs.items() if v["status"] != 0}
    if bad:
        print(json.dumps({"metric": "two-stage Jacobi", "error": f"solve status {bad}"}))
        sys.exit(1)
    best = min((k for k in runs if k != "fp64_only"), key=lambda k: runs[k]["ms"])
    dp = runs["fp64_only"]
    # algorithmic bytes of one iteration: values + columns, row pointers, and
    # x gathered once, b, diag(A) and x_{k+1}
    m = a.nnz
    byt64 = (8 + 4) * m + 4 * (n + 1) + 4 * 8 * n
    byt32 = (4 + 4) * m + 4 * (n + 1) + 4 * 4 * n
    it64_us, it32_us = kus["jacobi_f64"], kus["jacobi_f32"]
    out = {"metric": "two-stage Jacobi (Algorithm I with the Jacobi method): time to 1e-10, mixed vs FP64-only",
           "value": runs[best]["ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f32+f64",
           "config": {"workload": f"random banded n={n}, full bandwidth 17, density 0.8, Algorithm III values, mu=3, "
                                  "x~U(1,2), b=Ax, eps2=1e-10", "n": a.n, "m": a.nnz},
           "best_eps1": best, "fp64_only_ms": dp["ms"], "speedup_vs_fp64_only": round(dp["ms"] / runs[best]["ms"], 3),
           "iteration_f64": {"us": round(it64_us, 2), "bytes": byt64, "GBs": round(byt64 / it64_us / 1e3, 1),
                             "frac_hbm": round(byt64 / it64_us / 1e3 / 8000.0, 3)},
           "iteration_f32": {"us": round(it32_us, 2), "bytes": byt32, "GBs": round(byt32 / it32_us / 1e3, 1),
                             "frac_hbm": round(byt32 / it32_us / 1e3 / 8000.0, 3)},
           "runs": runs}
    print(json.dumps(out))


def bench_serve(args):
    """Poisson arrivals at ~80% of the measured saturation throughput; each
    request gets the feature pass and kNN eps1; the same arrival trace is
    replayed with FP64-only CG.  Requests draw their system from a pool of
    distinct systems (n log-uniform, four families) resident on the GPU, and
    write their solution into a buffer of their own until they are polled.
    Latency = completion (seen by polling) minus scheduled arrival."""
    import numpy as np
    import torch
    from paper_2412_08059_amd import DEFAULT_MODEL, BatchSolver, DeviceCSR
    t = time.perf_counter()
    pool = _mixed_systems(args.serve_pool, args.serve_nmin, args.serve_nmax, args.seed + 5000)
    prow = [((a.n + 63) // 64) * 64 for _, a, _ in pool]
    dev = [(DeviceCSR.from_host(a), torch.from_numpy(b).cuda()) for _, a, b in pool]
    fams = {f: sum(1 for g, _, _ in pool if g == f) for f in ("lap2d", "lap3d", "banded", "er")}
    count = args.serve_count
    rng = np.random.default_rng(args.seed + 7)
    which = rng.integers(0, len(pool), size=count)
    print(f"# serve: {count} requests over a pool of {len(pool)} systems ({sum(prow)} padded rows, "
          f"generated in {time.perf_counter() - t:.1f}s)", file=sys.stderr, flush=True)
    cap_rows = max(sum(prow) // 4, max(prow))
    cap_nnz = max(sum(a.nnz for _, a, _ in pool) // 2 + 64 * cap_rows, 2 * max(a.nnz for _, a, _ in pool) + 64 * cap_rows)
    eng = BatchSolver(cap_rows, cap_nnz, 256, model=DEFAULT_MODEL)
    free_x = {i: [] for i in range(len(pool))}

    def take_x(i):
        if free_x[i]:
            return free_x[i].pop()
        return torch.empty(pool[i][1].n, dtype=torch.float64, device="cuda")

    # saturation throughput: the first requests of the trace submitted at once
    ns = min(count, 2 * len(pool))
    xs = [take_x(int(which[k])) for k in range(ns)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = eng.wait_all(eng.submit([(dev[int(which[k])][0], dev[int(which[k])][1], xs[k], 0.0, 1e-10)
                                   for k in range(ns)]), timeout_s=3600)
    mu = ns / (time.perf_counter() - t0)
    for k in range(ns):
        free_x[int(which[k])].append(xs[k])
    lam = 0.8 * mu
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=count))
    print(f"# serve: saturation {mu:.2f} solves/s ({ns} requests at once), arrival rate {lam:.2f}/s",
          file=sys.stderr, flush=True)
    out_modes = {}
    for label, e1 in (("auto", 0.0), ("fp64_only", -1.0)):
        lat, done_t, occ, order = {}, {}, [], {}
        t0 = time.perf_counter()
        t_print = t0
        nxt = 0
        while len(done_t) < count:
            now = time.perf_counter() - t0
            batch = []
            while nxt < count and arrivals[nxt] <= now:
                batch.append(nxt)
                nxt += 1
            if batch:
                xb = [take_x(int(which[k])) for k in batch]
                ids = eng.submit([(dev[int(which[k])][0], dev[int(which[k])][1], x, e1, 1e-10)
                                  for k, x in zip(batch, xb)])
                for rid, k, x in zip(ids, batch, xb):
                    order[rid] = (k, x)
            for rid, st, _ in eng.poll():
                k, x = order.pop(rid)
                done_t[k] = time.perf_counter() - t0
                lat[k] = (done_t[k] - arrivals[k], st.status, st.relres_final_true)
                free_x[int(which[k])].append(x)
            q, a = eng.load()
            occ.append(a)
            if time.perf_counter() - t_print > 10.0:
                t_print = time.perf_counter()
                print(f"# serve {label}: {len(done_t)}/{count} done, {nxt} arrived, {a} active, {q} queued",
                      file=sys.stderr, flush=True)
            time.sleep(0.0005)
        L = np.array([v[0] for v in lat.values()]) * 1e3
        fails = sum(1 for v in lat.values() if v[1] != 0 or v[2] > 1e-10)
        span = max(done_t.values()) - arrivals[0]
        out_modes[label] = {"p50_ms": round(float(np.percentile(L, 50)), 1),
                            "p99_ms": round(float(np.percentile(L, 99)), 1),
                            "mean_ms": round(float(L.mean()), 1), "solves_per_s": round(count / span, 2),
                            "mean_active": round(float(np.mean(occ)), 2), "failed": fails}
        print(f"# serve {label}: {out_modes[label]}", file=sys.stderr, flush=True)
    eng.close()
    note = "" if count >= 10000 else f" ({count} of the configured 10,000 requests)"
    out = {"metric": "served solves: p50/p99 latency (arrival -> result) and solves/s", "value": out_modes["auto"]["p99_ms"],
           "unit": "ms (p99)", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": f"{count} Poisson-arrival requests{note} at 0.8 x saturation ({mu:.2f}/s), each "
                                  f"drawing one of {len(pool)} resident systems, n log-uniform "
                                  f"[{args.serve_nmin:g}, {args.serve_nmax:g}], families {fams}, eps2=1e-10",
                      "requests": count, "pool": len(pool), "arrival_rate_per_s": round(lam, 3)},
           "modes": out_modes}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--model", default=None, help="kNN model file (default: the packaged one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-jacobi", action="store_true", help="skip the Jacobi-preconditioned solves")
    ap.add_argument("--kernel-only", action="store_true",
                    help="for PMC runs: a 1 GiB device copy (counter calibration) and 20 launches of "
                         "each CG kernel on the workload, nothing else")
    ap.add_argument("--kernel-band", action="store_true",
                    help="with --kernel-only: the 4e6-row band (--large-n) instead of the 3D grid")
    ap.add_argument("--workload", choices=("solve", "batch", "serve", "family", "jacobi_iter", "diameter"),
                    default="solve",
                    help="solve: the 128^3 single-system benchmark (default); batch: many systems in one "
                         "engine; serve: Poisson arrivals with continuous admission; family: the paper's "
                         "kNN experiment on its three matrix families; jacobi_iter: Algorithm I with the Jacobi "
                         "method; diameter: the banded / random-graph contrast at n = 1M (features, kNN eps1 "
                         "against the swept optimum)")
    ap.add_argument("--jac-n", type=int, default=1 << 21)
    ap.add_argument("--family-n", type=int, default=1000)
    ap.add_argument("--family-scale", type=float, default=0.25, help="fraction of the appendix sample sizes")
    ap.add_argument("--family-reps", type=int, default=20)
    ap.add_argument("--family-no-omega", action="store_true", help="skip the per-matrix omega measurement")
    ap.add_argument("--dot-acc", type=int, default=0, choices=(0, 1),
                    help="family workload: FP32-phase dot products accumulated in FP64 (0) or FP32 (1)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-nmin", type=float, default=1e3)
    ap.add_argument("--batch-nmax", type=float, default=2e5)
    ap.add_argument("--large-n", type=int, default=4_000_000, help="rows of the >1 GB band case")
    ap.add_argument("--no-large", action="store_true", help="skip the >1 GB band kernel timings")
    ap.add_argument("--no-c1", action="store_true", help="skip the 2D Poisson 64^2 (C1) solves")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-pool", type=int, default=96, help="distinct resident systems the requests draw from")
    ap.add_argument("--serve-nmin", type=float, default=1e4)
    ap.add_argument("--serve-nmax", type=float, default=4e6)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the single-system solve "
              "is not sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "family":
        return bench_family(args)
    if args.workload == "jacobi_iter":
        return bench_jacobi_iter(args)
    if args.workload == "diameter":
        return bench_diameter(args)

    import numpy as np
    import torch

    import workloads as W
    from paper_2412_08059_amd import DEFAULT_MODEL, DeviceCSR, Solver, capi

    model = args.model or DEFAULT_MODEL
    have_model = os.path.exists(model)
    t_gen = time.perf_counter()
    if args.kernel_only and args.kernel_band:
        a = W.banded(args.large_n, 8, seed=args.seed)   # the >1 GB band, for counter runs
    else:
        a = W.varcoef3d(args.grid, seed=args.seed)
    xstar, b = W.rhs(a, seed=args.seed)
    t_gen = time.perf_counter() - t_gen
    n, m = a.n, a.nnz
    print(f"# workload varcoef3d {args.grid}^3 n={n} m={m} (generated in {t_gen:.1f}s); "
          f"model={'%s' % model if have_model else 'none (fixed eps1 1e-4)'}", file=sys.stderr, flush=True)

    solver = Solver(n, m, model=model if have_model else None)
    A = DeviceCSR.from_host(a)
    B = torch.from_numpy(b).cuda()
    if args.kernel_only:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        kus = {}
        for kname, kid in (("cg_spmv_f64", capi.MPCG_KERNEL_CG_SPMV_F64), ("update_f64", capi.MPCG_KERNEL_UPDATE_F64),
                           ("cg_spmv_f32", capi.MPCG_KERNEL_CG_SPMV_F32), ("update_f32", capi.MPCG_KERNEL_UPDATE_F32)):
            kus[kname] = round(capi.mpcg_time_kernel(solver.ctx, A.desc, kid, 20) * 1e3, 2)
        solver.close()
        print(json.dumps({"kernel_only": True, "copy_bytes": 1 << 30, "us_per_launch": kus}))
        return
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    XD = torch.empty(n, dtype=torch.float64, device="cuda")
    eps1 = capi.MPCG_EPS1_AUTO if have_model else 1e-4
    torch.cuda.synchronize()

    def step():
        t0 = time.perf_counter()
        st1, _, sm = solver.solve(A, B, eps1, 1e-10, x=X)
        t1 = time.perf_counter()
        st2, _, sd = solver.solve(A, B, capi.MPCG_EPS1_NONE, 1e-10, x=XD)
        t2 = time.perf_counter()
        if st1 != 0 or st2 != 0:
            raise RuntimeError(f"solve failed: mixed {st1}, fp64-only {st2}")
        if sm.relres_final_true > 1e-10 or sd.relres_final_true > 1e-10:
            raise RuntimeError("final residual above eps2")
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, sm, sd

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mixed, dp = [], []
    T0 = time.perf_counter()
    for k in range(args.steps):
        tm, td, sm, sd = step()
        mixed.append(tm)
        dp.append(td)
        print(f"# step {k}: mixed {tm:.1f} ms (N1={sm.n1}, N2={sm.n2}, eps1={sm.eps1_used:g}, "
              f"feat {sm.t_feat_ms:.1f} ms), fp64-only {td:.1f} ms (N_dp={sd.n2})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    ms_per_step = (T1 - T0) * 1e3 / args.steps
    mixed_ms = float(np.mean(mixed))
    dp_ms = float(np.mean(dp))
    x_mixed = X.cpu().numpy().copy()
    x_dp = XD.cpu().numpy().copy()
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
    err_xstar = {"mixed": rel(x_mixed, xstar), "fp64_only": rel(x_dp, xstar)}

    # per-kernel launch times, HIP events on the library stream
    reps = 30
    kern = {
        "cg_spmv_f64": capi.MPCG_KERNEL_CG_SPMV_F64, "cg_spmv_f32": capi.MPCG_KERNEL_CG_SPMV_F32,
        "update_f64": capi.MPCG_KERNEL_UPDATE_F64, "update_f32": capi.MPCG_KERNEL_UPDATE_F32,
        "spmv_f64": capi.MPCG_KERNEL_SPMV_F64, "spmv_f32": capi.MPCG_KERNEL_SPMV_F32,
    }
    kt = {k: capi.mpcg_time_kernel(solver.ctx, A.desc, v, reps) for k, v in kern.items()}
    kernels = {}
    for k, ms in kt.items():
        byt = kernel_bytes(k, n, m)
        fbyt = sell_format_bytes(k, a)
        kernels[k] = {"us": round(ms * 1e3, 2), "GBs": round(byt / (ms * 1e-3) / 1e9, 1),
                      "bytes": int(byt), "format_bytes": int(fbyt),
                      "frac_format": round(fbyt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    # dominant kernel of the mixed step = largest launch count x duration
    share = {"cg_spmv_f32": sm.n1 * kt["cg_spmv_f32"], "update_f32": sm.n1 * kt["update_f32"],
             "cg_spmv_f64": sm.n2 * kt["cg_spmv_f64"], "update_f64": sm.n2 * kt["update_f64"]}
    dom = max(share, key=share.get)
    dom_gbs = kernels[dom]["GBs"]
    traffic = measured_traffic(dom, f"varcoef3d {args.grid}^3 seed {args.seed}")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_gbs / HBM_PEAK_GBS, 3),
                "traffic": None if traffic is None else int(traffic),
                "bytes_per_launch": kernels[dom]["bytes"], "us_per_launch": kernels[dom]["us"],
                "format_bytes_per_launch": kernels[dom]["format_bytes"],
                "frac_format": kernels[dom]["frac_format"],
                "working_set_under_256MB_infinity_cache": kernels[dom]["format_bytes"] < 256e6}

    sweep = None
    if not args.no_sweep:
        sweep = []
        for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
            t0 = time.perf_counter()
            st, _, s = solver.solve(A, B, e, 1e-10, x=X)
            t1 = time.perf_counter()
            sweep.append({"eps1": e, "ms": round((t1 - t0) * 1e3, 1), "n1": s.n1, "n2": s.n2, "status": st})
        best = min(sweep, key=lambda r: r["ms"])
        print(f"# eps1 sweep: " + ", ".join(f"{r['eps1']:g}:{r['ms']}ms({r['n1']}/{r['n2']})" for r in sweep)
              + f"; best {best['eps1']:g}", file=sys.stderr, flush=True)

    # Jacobi-preconditioned stages on the same system (reported beside the
    # headline, which is the paper's unpreconditioned method)
    jac = None
    if not args.no_jacobi:
        sj = Solver(n, m, model=model if have_model else None, precond=1)
        jr = {}
        for label, e in (("mixed", eps1), ("fp64_only", capi.MPCG_EPS1_NONE)):
            sj.solve(A, B, e, 1e-10, x=X)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _, sj_s = sj.solve(A, B, e, 1e-10, x=X)
            torch.cuda.synchronize()
            jr[label] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "n1": sj_s.n1, "n2": sj_s.n2,
                         "status": st, "relres_final_true": sj_s.relres_final_true,
                         "eps1": sj_s.eps1_used}
        sj.close()
        jac = {"mixed_ms": jr["mixed"]["ms"], "fp64_only_ms": jr["fp64_only"]["ms"],
               "speedup_vs_fp64_only": round(jr["fp64_only"]["ms"] / jr["mixed"]["ms"], 3), "runs": jr}
        print(f"# jacobi: {jac}", file=sys.stderr, flush=True)

    c1 = None if args.no_c1 else bench_c1(args)
    if c1 is not None:
        print(f"# C1 Poisson 64^2: {json.dumps(c1)}", file=sys.stderr, flush=True)
    large = None if args.no_large else bench_large_band(args)
    if large is not None:
        print(f"# large band: {json.dumps(large)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(a, b, model, x_mixed, x_dp, sm.n1, sm.n2, sd.n2)
        print(f"# cpu baseline: {json.dumps(cpu)}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(mixed_ms, 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point variable-coefficient diffusion {args.grid}^3, face coefficients "
                               f"10^U(0,3), x*~U[-1,1] seed {args.seed}, b=Ax*, eps2=1e-10",
                   "n": n, "m": m, "eps1_mode": "auto (2BFS + v + kNN)" if have_model else "fixed 1e-4"},
        "fp64_only_ms": round(dp_ms, 2),
        "speedup_vs_fp64_only": round(dp_ms / mixed_ms, 3),
        "n1": sm.n1, "n2": sm.n2, "n_dp": sd.n2, "eps1": sm.eps1_used, "eps1_class": sm.eps1_class,
        "pdiam": sm.feat.pdiam, "v": round(sm.feat.v, 6), "t_feat_ms": round(sm.t_feat_ms, 3),
        "feat_frac_of_fp64_only": round(sm.t_feat_ms / dp_ms, 4),
        "omega_measured": round(sm.omega_measured, 3),
        "I_third": round(sm.I_third, 2), "I_meas": round(sm.I_meas, 2),
        "equiv_fp64_iters_per_s": round(sd.n2 / (mixed_ms * 1e-3), 1),
        "relres_final_true": sm.relres_final_true,
        "spmv_f64_GBs": kernels["spmv_f64"]["GBs"],
        "spmv_frac_hbm": round(kernels["spmv_f64"]["GBs"] / HBM_PEAK_GBS, 3),
        "cg_spmv_f64_frac_hbm": round(kernels["cg_spmv_f64"]["GBs"] / HBM_PEAK_GBS, 3),
        "err_vs_xstar": err_xstar,
        "err_vs_oracle": None if cpu is None else cpu["err_vs_oracle"],
        "kappa_hat": None if cpu is None else cpu["kappa_hat"],
        "kernels": kernels,
        "c1_poisson2d_64": c1,
        "large_band": large,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "eps1_sweep": sweep,
        "jacobi": jac,
    }
    solver.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
