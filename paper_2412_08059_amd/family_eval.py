"""The paper's kNN experiment (its "Computational Experiments" section and the
appendix on samples, training/test formation and efficiency), run on this GPU.

For every matrix of a general sample S0:
  * its features (n, m, 2BFS pseudo-diameter, v over k0 = 20 FP32
    iterations) and, for each eps1 = 10^-t (t = 2..7) and for FP64-only CG,
    the iteration counts N1, N2 -- all through the batch engine;
  * the optimal class t^ = argmin_t I_t, I_t = omega N1(t) + N2(t) (eq. 4,
    ties to the larger eps1) with omega = 1/3.

Then, over repeated random splits of S0 into a training set S of the size
eq. 26 gives (alpha = 0.01, c = 0.1, k_CG = the mean FP64-only iteration
count over S0) and the test set T = S0 \\ S, the library's kNN -- a model file
written from the training rows, with the paper's experimental feature set
(m, pseudo-diameter, v) -- classifies every test matrix, and:
  * Acc  = share of test matrices classified into their optimal class;
  * Loc  = mean share of same-class rows among a test matrix's k nearest
           training rows (the paper's localisation measure);
  * E, E_opt of eq. 27 over T, for omega = 1/3 and for the matrix's measured
    omega (ratio of FP32 to FP64 CG-iteration kernel time on this GPU); as in
    the paper, the classes stay the omega = 1/3 ones and only the cost
    accounting changes with omega;
  * and, for this GPU, the same with the classes re-optimised for the
    measured omega (a second classifier trained on those classes).
Means and standard deviations over the splits are reported.
"""

from __future__ import annotations

import math
import os
import tempfile
import time

import numpy as np

EPS1 = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7)
KS = (1, 5, 10, 15, 20)
MASK = 14   # (m, pseudo-diameter, v)


def training_size(n: float, k_cg: float, k: int, alpha: float = 0.01, c: float = 0.1) -> float:
    """N_S of eq. 26 as the appendix uses it."""
    return alpha * 4.0 * (6.0 * c + 17.0) * n * k_cg / (44.0 + 3.0 * k)


def costs(n1: np.ndarray, n2: np.ndarray, omega) -> np.ndarray:
    """I_t = omega * N1(t) + N2(t), shape (N, 6); omega scalar or per row."""
    w = np.asarray(omega, dtype=np.float64)
    if w.ndim == 1:
        w = w[:, None]
    return w * n1 + n2


def optimal_class(I: np.ndarray) -> np.ndarray:
    """2 + argmin over the six classes (first -- larger eps1 -- on ties)."""
    return 2 + np.argmin(I, axis=1)


def efficiency(I_sel: np.ndarray, I_dp: np.ndarray) -> float:
    """eq. 27: (1 - sum I / sum I_dp) * 100."""
    return (1.0 - float(np.sum(I_sel)) / float(np.sum(I_dp))) * 100.0


def _norm01(x, lo, hi):
    span = hi - lo
    out = np.zeros_like(x, dtype=np.float64)
    ok = span > 0
    out[..., ok] = (x[..., ok] - lo[ok]) / span[ok]
    return out


def localization(ftr: np.ndarray, ltr: np.ndarray, fte: np.ndarray, lte: np.ndarray, k: int,
                 mask: int = MASK) -> float:
    """Mean fraction (percent) of same-class rows among each test row's k
    nearest training rows: min-max scaling over the training rows, squared
    Euclidean distance over the masked features, ties to the lower index."""
    cols = [j for j in range(4) if mask & (1 << j)]
    lo = ftr.min(axis=0)
    hi = ftr.max(axis=0)
    a = _norm01(ftr, lo, hi)[:, cols]
    q = _norm01(fte, lo, hi)[:, cols]
    kk = min(k, len(ftr))
    frac = np.empty(len(fte))
    for s in range(0, len(fte), 512):
        d2 = ((q[s:s + 512, None, :] - a[None, :, :]) ** 2).sum(axis=2)
        nn = np.argsort(d2, axis=1, kind="stable")[:, :kk]
        frac[s:s + 512] = (ltr[nn] == lte[s:s + 512, None]).mean(axis=1)
    return float(frac.mean() * 100.0)


def write_model(path: str, feat: np.ndarray, lab: np.ndarray, k: int, mask: int = MASK, omega: float = 1 / 3):
    with open(path, "w") as f:
        f.write("mpcg-knn-model 1\n")
        f.write(f"k {int(k)}\nmask {int(mask)}\nomega {omega:.17g}\nns {len(lab)}\n")
        f.write("fmin " + " ".join(f"{v:.17g}" for v in feat.min(axis=0)) + "\n")
        f.write("fmax " + " ".join(f"{v:.17g}" for v in feat.max(axis=0)) + "\n")
        for row, t in zip(feat, lab):
            f.write(" ".join(f"{v:.17g}" for v in row) + f" {int(t)}\n")


# ------------------------------------------------------------ GPU labelling --

def label(matrices, rhs_fn, engine, eps2: float = 1e-10, chunk: int = 128, omega_solver=None,
          omega_launches: int = 10):
    """Features and per-class iteration counts of every matrix through the
    batch engine (one Algorithm II request for the features, six Algorithm I
    requests and one FP64-only request per matrix).  `rhs_fn(a, i)` gives b.
    Returns one dict per matrix and the wall time in seconds."""
    import torch
    from . import DeviceCSR, capi

    rows = []
    t0 = time.perf_counter()
    modes = (0.0,) + EPS1 + (-1.0,)
    for s in range(0, len(matrices), chunk):
        part = matrices[s:s + chunk]
        reqs, keep = [], []
        for i, a in enumerate(part):
            b = rhs_fn(a, s + i)
            A = DeviceCSR.from_host(a)
            B = torch.from_numpy(b).cuda()
            for e in modes:
                X = torch.empty(a.n, dtype=torch.float64, device="cuda")
                reqs.append((A, B, X, e, eps2))
            keep.append(A)
        ids = engine.submit(reqs)
        got = engine.wait_all(ids, timeout_s=600)
        for i, a in enumerate(part):
            st = [got[ids[i * len(modes) + j]][0] for j in range(len(modes))]
            bad = [x.status for x in st if x.status != 0]
            if bad:
                raise RuntimeError(f"matrix {s + i} ({a.name}): status {bad}")
            f = st[0].feat
            r = dict(name=a.name, n=int(f.n), m=int(f.m), pdiam=int(f.pdiam), v=float(f.v),
                     bfs_t=int(f.bfs_t), bfs_u=int(f.bfs_u), ncomp=int(f.n_components),
                     n1=[int(x.n1) for x in st[1:7]], n2=[int(x.n2) for x in st[1:7]],
                     flags=[int(x.flags) for x in st[1:7]], n_dp=int(st[7].n2))
            if omega_solver is not None:
                r["omega"] = measured_omega(omega_solver, keep[i], omega_launches)
            rows.append(r)
    torch.cuda.synchronize()
    return rows, time.perf_counter() - t0


def measured_omega(solver, A, launches: int = 10) -> float:
    """Ratio of the FP32 to the FP64 CG-iteration kernel time (product +
    update) on this GPU for matrix A."""
    from . import capi
    t32 = (capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_CG_SPMV_F32, launches)
           + capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_UPDATE_F32, launches))
    t64 = (capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_CG_SPMV_F64, launches)
           + capi.mpcg_time_kernel(solver.ctx, A.desc, capi.MPCG_KERNEL_UPDATE_F64, launches))
    return t32 / t64


# -------------------------------------------------------------- evaluation --

def _classify(ctx, path: str, fte: np.ndarray) -> np.ndarray:
    from . import capi
    st = capi.mpcg_load_model(ctx, path)
    if st != 0:
        raise RuntimeError(f"mpcg_load_model status {st}")
    out = np.empty(len(fte), dtype=np.int64)
    f = capi.mpcg_features_t()
    for i, row in enumerate(fte):
        f.n, f.m, f.pdiam, f.v = int(row[0]), int(row[1]), int(row[2]), float(row[3])
        st, _, cls = capi.mpcg_select_eps1(ctx, f)
        if st != 0:
            raise RuntimeError(f"mpcg_select_eps1 status {st}")
        out[i] = cls
    return out


def evaluate(rows, ks=KS, reps: int = 20, seed: int = 0, mask: int = MASK):
    """Acc, Loc, E and E_opt (omega = 1/3 and measured omega) per k, as means
    and standard deviations over `reps` random training/test splits."""
    import torch
    from . import capi

    N = len(rows)
    feat = np.array([[r["n"], r["m"], r["pdiam"], r["v"]] for r in rows], dtype=np.float64)
    n1 = np.array([r["n1"] for r in rows], dtype=np.float64)
    n2 = np.array([r["n2"] for r in rows], dtype=np.float64)
    ndp = np.array([r["n_dp"] for r in rows], dtype=np.float64)
    have_om = all("omega" in r for r in rows)
    om = np.array([r.get("omega", 1 / 3) for r in rows], dtype=np.float64)
    I3 = costs(n1, n2, 1.0 / 3.0)
    lab = optimal_class(I3)
    Im = costs(n1, n2, om)
    lab_m = optimal_class(Im)   # classes re-optimised for the measured omega
    k_cg = float(ndp.mean())
    n_size = float(np.median(feat[:, 0]))
    dist = {f"1e-{t}": round(float(np.mean(lab == t) * 100.0), 1) for t in range(2, 8)}
    dist_m = {f"1e-{t}": round(float(np.mean(lab_m == t) * 100.0), 1) for t in range(2, 8)}
    ctx = capi.mpcg_create(None, torch.cuda.current_stream().cuda_stream)
    out = dict(N=N, k_CG=round(k_cg, 2), class_distribution_pct=dist,
               class_distribution_meas_pct=dist_m if have_om else None,
               omega_measured_median=round(float(np.median(om)), 4) if have_om else None, per_k={})
    rng = np.random.default_rng(seed)
    try:
        with tempfile.TemporaryDirectory() as tmp:
            for k in ks:
                ns = int(round(training_size(n_size, k_cg, k)))
                ns = max(k, min(ns, N - 1))
                acc, loc, e3, e3o, em, emo, accr, err, erro = [], [], [], [], [], [], [], [], []
                for r in range(reps):
                    perm = rng.permutation(N)
                    tr, te = perm[:ns], perm[ns:]
                    path = os.path.join(tmp, f"m_{k}_{r}.txt")
                    write_model(path, feat[tr], lab[tr], k, mask)
                    cls = _classify(ctx, path, feat[te])
                    sel = cls - 2
                    acc.append(float(np.mean(cls == lab[te]) * 100.0))
                    loc.append(localization(feat[tr], lab[tr], feat[te], lab[te], k, mask))
                    opt = lab[te] - 2
                    ti = np.arange(len(te))
                    e3.append(efficiency(I3[te][ti, sel], ndp[te]))
                    e3o.append(efficiency(I3[te][ti, opt], ndp[te]))
                    em.append(efficiency(Im[te][ti, sel], ndp[te]))
                    emo.append(efficiency(Im[te][ti, opt], ndp[te]))
                    if have_om:   # a classifier trained on the measured-omega classes
                        write_model(path, feat[tr], lab_m[tr], k, mask)
                        clr = _classify(ctx, path, feat[te])
                        accr.append(float(np.mean(clr == lab_m[te]) * 100.0))
                        err.append(efficiency(Im[te][ti, clr - 2], ndp[te]))
                        erro.append(efficiency(Im[te][ti, lab_m[te] - 2], ndp[te]))

                def ms(v):
                    return [round(float(np.mean(v)), 2), round(float(np.std(v)), 2)]

                out["per_k"][str(k)] = dict(N_S=ns, N_T=N - ns, Acc=ms(acc), Loc=ms(loc), E_third=ms(e3),
                                            E_opt_third=ms(e3o),
                                            E_meas=ms(em) if have_om else None,
                                            E_opt_meas=ms(emo) if have_om else None,
                                            relabelled_meas=dict(Acc=ms(accr), E=ms(err), E_opt=ms(erro))
                                            if have_om else None)
    finally:
        capi.mpcg_destroy(ctx)
    return out
