"""GPU parity of the paper-family experiment: features and per-eps1 iteration
counts of the three matrix families through the batch engine against the
oracle, the optimal class, and the train/test evaluation end to end through
the library's kNN.

Bars: pseudo-diameter, t, u and component count bit-exact; v within 1e-9;
N1, N2 per eps1 and the FP64-only count within max(1, ceil(5 %)) of the
oracle's (an FP32 phase that stops at its iteration cap on either side is not
compared: near the FP32 rounding floor the crossing iteration is not
determined by the arithmetic); the optimal class equal to the oracle's
wherever the oracle's best cost beats the runner-up by more than 10 %."""

import math

import numpy as np
import pytest

import oracle
from workloads import paper_family as PF

pytestmark = pytest.mark.gpu

EPS2 = 1e-10
FAMS = [("star", 301), ("random", 300), ("banded", 300)]


@pytest.fixture(scope="module")
def engine():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2412_08059_amd import BatchSolver, DEFAULT_MODEL
    e = BatchSolver(300_000, 6_000_000, 64, model=DEFAULT_MODEL)
    yield e
    e.close()


def band_ok(n_gpu, n_or):
    return abs(n_gpu - n_or) <= max(1, math.ceil(0.05 * n_or))


def _sample(fam, n, count, seed):
    specs = PF.sample_specs(fam, n)
    rng = np.random.default_rng(seed)
    pick = sorted(rng.choice(len(specs), size=count, replace=False).tolist())
    return [PF.make(specs[i]) for i in pick]


def _rhs(a, i):
    return PF.paper_rhs(a, 500 + i)[1]


@pytest.mark.parametrize("fam,n", FAMS)
def test_family_labels_match_oracle(engine, fam, n):
    from paper_2412_08059_amd import capi, family_eval as FE
    mats = _sample(fam, n, 8, seed=3)
    print(f"family {fam} n={n}: {len(mats)} matrices", flush=True)
    rows, _ = FE.label(mats, _rhs, engine, eps2=EPS2)
    dummy = oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1]]), [2], k=1)
    for i, (a, r) in enumerate(zip(mats, rows)):
        b = _rhs(a, i)
        assert (r["pdiam"], r["bfs_t"], r["bfs_u"], r["ncomp"]) == oracle.pseudo_diameter(a), a.name
        ra = oracle.solve(a, b, oracle.EPS1_AUTO, EPS2, model=dummy)
        assert abs(r["v"] - ra.v) <= 1e-9 * max(1.0, abs(ra.v)), a.name
        n1o, n2o = [], []
        for t, e in enumerate(FE.EPS1):
            ro = oracle.solve(a, b, e, EPS2)
            assert ro.status == 0
            n1o.append(ro.n1)
            n2o.append(ro.n2)
            capped = (ro.flags | r["flags"][t]) & capi.MPCG_FLAG_FP32_MAXIT
            if not capped:
                assert band_ok(r["n1"][t], ro.n1), (a.name, e, r["n1"][t], ro.n1)
                assert band_ok(r["n2"][t], ro.n2), (a.name, e, r["n2"][t], ro.n2)
        rdp = oracle.solve(a, b, -1.0, EPS2)
        assert band_ok(r["n_dp"], rdp.n2), (a.name, r["n_dp"], rdp.n2)
        I = FE.costs(np.array([n1o], float), np.array([n2o], float), 1 / 3)[0]
        srt = np.sort(I)
        if srt[1] > 1.1 * srt[0]:
            Ig = FE.costs(np.array([r["n1"]], float), np.array([r["n2"]], float), 1 / 3)
            assert FE.optimal_class(Ig)[0] == 2 + int(np.argmin(I)), a.name


def test_family_evaluation_end_to_end(engine):
    """Labelling, splits, the library's kNN on each split's model file, and
    the eq. 27 accounting, on a small random-family sample."""
    from paper_2412_08059_amd import Solver, family_eval as FE
    mats = _sample("random", 300, 40, seed=5)
    solver = Solver(400, 12_000)
    rows, secs = FE.label(mats, _rhs, engine, eps2=EPS2, omega_solver=solver)
    solver.close()
    assert len(rows) == 40 and secs > 0
    res = FE.evaluate(rows, ks=(1, 5), reps=3, seed=1)
    assert res["N"] == 40 and abs(sum(res["class_distribution_pct"].values()) - 100.0) < 0.5
    for k, r in res["per_k"].items():
        assert r["N_S"] + r["N_T"] == 40
        assert 0.0 <= r["Acc"][0] <= 100.0 and 0.0 <= r["Loc"][0] <= 100.0
        # the optimal class is never worse than the chosen one
        assert r["E_opt_third"][0] >= r["E_third"][0] - 1e-9
        assert r["E_meas"] is not None
