"""GPU parity at the workloads' full sizes and on the final-check restart,
through the C ABI, against the CPU oracle on the same seeded inputs.

Bars (the parity bars of the single solves):
  * status OK and the final true relative residual <= eps2 on both sides;
  * iteration counts per phase within max(1, ceil(5 %)) of the oracle's;
  * ||x_gpu - x_or|| / ||x_or|| <= 1e-8 when the oracle's CG-Lanczos estimate
    kappa-hat is at most 1e6, else within 2 kappa-hat eps2 (the distance two
    solutions that both meet eps2 may have);
  * Algorithm II: pseudo-diameter, t, u bit-exact, v within 1e-9, and the kNN
    class equal both to the oracle selector's on the GPU's features and to
    the oracle's own class.

The oracle runs its row loops on the host's threads (the same bits as one
thread) so that a 2M-row solve finishes in tens of seconds."""

import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TEST_MODEL = os.path.join(GOLDEN, "knn_model_test.txt")
PKG_MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2412_08059_amd",
                         "knn_model.txt")
EPS2 = 1e-10
RESTART_EPS2 = 3e-12


def band_ok(n_gpu, n_or):
    return abs(n_gpu - n_or) <= max(1, math.ceil(0.05 * n_or))


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    oracle.set_threads(_threads())
    yield torch
    oracle.set_threads(1)


@pytest.fixture(scope="module")
def solver(torch_mod):
    from paper_2412_08059_amd import Solver
    s = Solver(2_200_000, 17_500_000, model=PKG_MODEL)
    yield s
    s.close()


def dev(a):
    from paper_2412_08059_amd import DeviceCSR
    return DeviceCSR.from_host(a)


def t64(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_x(xg, r, kappa, eps2=EPS2):
    d = rel(xg, r.x)
    bar = 1e-8 if kappa <= 1e6 else 2.0 * kappa * eps2
    assert d <= bar, (d, bar, kappa)
    return d


# ------------------------------------------------------ final-check restart --

@pytest.fixture(scope="module")
def restart_case():
    a = W.banded(20000, 8, seed=1, shift=1e-4)
    xs, b = W.smooth_rhs(a)
    return a, xs, b


@pytest.mark.parametrize("eps1", [-1.0, 1e-4])
def test_final_restart_parity(solver, torch_mod, restart_case, eps1):
    """The recursive residual reaches eps2 = 3e-12 while the true residual is
    about seven times larger (oracle), so the final check fails and CG starts
    again from x with r = b - Ax.  Both sides must restart and then meet
    eps2."""
    a, xs, b = restart_case
    print(f"final-restart case band 20000 shift 1e-4 smooth x*, eps1={eps1}", flush=True)
    st, x, s = solver.solve(dev(a), t64(torch_mod, b), eps1, RESTART_EPS2)
    r = oracle.solve(a, b, eps1, RESTART_EPS2)
    print(f"  gpu n1={s.n1} n2={s.n2} restarts={s.restarts} final={s.relres_final_true:.3e}; "
          f"oracle n1={r.n1} n2={r.n2} restarts={r.restarts} final={r.relres_final_true:.3e}", flush=True)
    from paper_2412_08059_amd import capi
    assert st == 0 and r.status == 0
    assert r.flags & oracle.FLAG_FINAL_RESTARTED and r.restarts >= 1
    assert s.flags & capi.MPCG_FLAG_FINAL_RESTARTED and s.restarts >= 1
    assert s.relres_final_true <= RESTART_EPS2
    assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2), ((s.n1, s.n2), (r.n1, r.n2))
    check_x(x.cpu().numpy(), r, 1.36e5, RESTART_EPS2)


def test_batch_final_restart_parity(torch_mod, restart_case):
    """The same restart inside the batch engine (the Resid -> Restart
    transition of a system's state machine), beside a system that does not
    restart."""
    from paper_2412_08059_amd import BatchSolver, capi, DeviceCSR
    a, xs, b = restart_case
    p = W.poisson2d(48)
    _, bp = W.rhs(p, seed=2)
    eng = BatchSolver(100_000, 1_000_000, 8, model=TEST_MODEL)
    try:
        sysd = []
        for m, rhs, e1, e2 in ((a, b, -1.0, RESTART_EPS2), (a, b, 1e-4, RESTART_EPS2), (p, bp, 1e-4, EPS2)):
            X = torch_mod.full((m.n,), float("nan"), dtype=torch_mod.float64, device="cuda")
            sysd.append((DeviceCSR.from_host(m), t64(torch_mod, rhs), X, e1, e2))
        ids = eng.submit(sysd)
        got = eng.wait_all(ids, timeout_s=100)
    finally:
        eng.close()
    for rid, (m, rhs, e1, e2) in zip(ids, ((a, b, -1.0, RESTART_EPS2), (a, b, 1e-4, RESTART_EPS2),
                                           (p, bp, 1e-4, EPS2))):
        s, X = got[rid]
        r = oracle.solve(m, rhs, e1, e2)
        print(f"batch n={m.n} eps1={e1}: gpu n1={s.n1} n2={s.n2} restarts={s.restarts}; "
              f"oracle {r.n1}/{r.n2}/{r.restarts}", flush=True)
        assert s.status == 0 and r.status == 0
        assert s.relres_final_true <= e2
        assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2)
        if m is a:
            assert s.flags & capi.MPCG_FLAG_FINAL_RESTARTED and r.flags & oracle.FLAG_FINAL_RESTARTED
        check_x(X.cpu().numpy(), r, 1.36e5, e2)


# ------------------------------------------- 3D varcoef 128^3 (the bench) --

@pytest.fixture(scope="module")
def varcoef128(torch_mod):
    a = W.varcoef3d(128, seed=0)
    xs, b = W.rhs(a, seed=0)
    return a, xs, b, dev(a), t64(torch_mod, b)


@pytest.fixture(scope="module")
def kappa128(varcoef128):
    a, xs, b, _, _ = varcoef128
    kap, lmin, lmax, k = oracle.lanczos_kappa(a, b, EPS2)
    print(f"varcoef3d 128^3: kappa-hat {kap:.4g} (lambda {lmin:.4g} .. {lmax:.4g}, {k} CG steps)", flush=True)
    return kap


@pytest.mark.parametrize("eps1", [-1.0, 1e-6])
def test_full_size_varcoef128_solve_parity(solver, torch_mod, varcoef128, kappa128, eps1):
    a, xs, b, A, B = varcoef128
    print(f"full varcoef3d 128^3 n={a.n} nnz={a.nnz} eps1={eps1}", flush=True)
    st, x, s = solver.solve(A, B, eps1, EPS2)
    xg = x.cpu().numpy()
    r = oracle.solve(a, b, eps1, EPS2)
    d = check_x(xg, r, kappa128)
    print(f"  gpu n1={s.n1} n2={s.n2} oracle n1={r.n1} n2={r.n2} |x-x_or|/|x_or|={d:.2e} "
          f"|x-x*|/|x*|={rel(xg, xs):.2e} oracle |x-x*|/|x*|={rel(r.x, xs):.2e}", flush=True)
    assert st == 0 and r.status == 0
    assert s.relres_final_true <= EPS2
    assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2), ((s.n1, s.n2), (r.n1, r.n2))


def test_full_size_varcoef128_auto_parity(solver, torch_mod, varcoef128, kappa128):
    """Algorithm II with the packaged kNN model, as the bench runs it."""
    a, xs, b, A, B = varcoef128
    model = oracle.load_model(PKG_MODEL)
    print(f"full varcoef3d 128^3 auto", flush=True)
    st, x, s = solver.solve(A, B, 0.0, EPS2)
    xg = x.cpu().numpy()
    r = oracle.solve(a, b, oracle.EPS1_AUTO, EPS2, model=model)
    f = s.feat
    print(f"  gpu class={s.eps1_class} n1={s.n1} n2={s.n2} v={f.v:.12f}; oracle class={r.eps1_class} "
          f"n1={r.n1} n2={r.n2} v={r.v:.12f}", flush=True)
    assert st == 0 and r.status == 0
    assert (f.pdiam, f.bfs_t, f.bfs_u) == (r.ell, r.bfs_t, r.bfs_u) == (381, a.n - 1, 0)
    assert abs(f.v - r.v) <= 1e-9
    t_sel, _, _ = oracle.knn_select(model, [f.n, f.m, f.pdiam, f.v])
    assert s.eps1_class == t_sel == r.eps1_class
    assert s.relres_final_true <= EPS2
    assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2), ((s.n1, s.n2), (r.n1, r.n2))
    check_x(xg, r, kappa128)


# ------------------------------------------------------- the n = 1M graphs --

def test_full_size_er_1M_solve_parity(solver, torch_mod):
    a = W.er_laplacian(1_000_000, 16, seed=0)
    xs, b = W.rhs(a, seed=0)
    A, B = dev(a), t64(torch_mod, b)
    model = oracle.load_model(PKG_MODEL)
    kap = oracle.lanczos_kappa(a, b, EPS2)[0]
    for e in (-1.0, 1e-5, 0.0):
        print(f"full er 1M eps1={e} (kappa-hat {kap:.3g})", flush=True)
        st, x, s = solver.solve(A, B, e, EPS2)
        r = oracle.solve(a, b, e, EPS2, model=model if e == 0.0 else None)
        assert st == 0 and r.status == 0
        assert s.relres_final_true <= EPS2
        assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2), ((s.n1, s.n2), (r.n1, r.n2))
        if e == 0.0:
            f = s.feat
            assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == (r.ell, r.bfs_t, r.bfs_u, r.ncomp)
            assert abs(f.v - r.v) <= 1e-9
            assert s.eps1_class == r.eps1_class == oracle.knn_select(model, [f.n, f.m, f.pdiam, f.v])[0]
        check_x(x.cpu().numpy(), r, kap)


def test_full_size_band_1M_solve_parity(solver, torch_mod):
    """The deep band at the class the packaged model picks for it (1e-7)."""
    a = W.banded(1_000_000, 8, seed=0)
    xs, b = W.rhs(a, seed=0)
    print("full band 1M eps1=1e-7", flush=True)
    st, x, s = solver.solve(dev(a), t64(torch_mod, b), 1e-7, EPS2)
    r = oracle.solve(a, b, 1e-7, EPS2)
    print(f"  gpu n1={s.n1} n2={s.n2} oracle n1={r.n1} n2={r.n2}", flush=True)
    assert st == 0 and r.status == 0
    assert s.relres_final_true <= EPS2
    assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2), ((s.n1, s.n2), (r.n1, r.n2))
    # kappa of this band is about 1.35e5 (shift 1e-4)
    check_x(x.cpu().numpy(), r, 1.35e5)
