"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars:
  * SpMV: bit-exact (both sides run one fma chain per row in CSR order).
  * BFS distances, 2BFS pseudo-diameter (t, u, components), kNN class on the
    same features: bit-exact.
  * CG solves: final true relative residual <= eps2; iteration counts per
    phase within max(1, ceil(5%)) of the oracle's; ||x_gpu - x_or|| / ||x_or||
    <= 1e-8 (dot-product summation order is the only arithmetic difference).
"""

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TEST_MODEL = os.path.join(GOLDEN, "knn_model_test.txt")


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


@pytest.fixture(scope="module")
def solver(torch_mod):
    from paper_2412_08059_amd import Solver
    s = Solver(2_200_000, 17_500_000, model=TEST_MODEL)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver_csr(torch_mod):
    """A context that always takes the CSR-stream kernels (the fallback used
    when the SELL-64 copy would need too much padding)."""
    from paper_2412_08059_amd import Solver
    s = Solver(200_000, 4_000_000, model=TEST_MODEL, spmv_variant=3)
    yield s
    s.close()


@pytest.fixture(params=["sell", "csr"])
def any_solver(request, solver, solver_csr):
    return solver if request.param == "sell" else solver_csr


@pytest.fixture(scope="module")
def solver_persist(torch_mod):
    """A context whose 2BFS expands large levels in one persistent launch
    (grid barrier between levels) instead of one launch per level."""
    from paper_2412_08059_amd import Solver
    s = Solver(2_200_000, 17_500_000, model=TEST_MODEL, bfs_mode=2)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver_dia(torch_mod):
    """A context whose 2BFS sweeps run as bit-parallel levels over the
    diagonals whenever the pattern lies on at most 16 of them."""
    from paper_2412_08059_amd import Solver
    s = Solver(2_200_000, 17_500_000, model=TEST_MODEL, tuning={"bfs_dia": 2})
    yield s
    s.close()


@pytest.fixture(params=["level", "persist", "dia"])
def bfs_solver(request, solver, solver_persist, solver_dia):
    return {"level": solver, "persist": solver_persist, "dia": solver_dia}[request.param]


def dev(a, **kw):
    from paper_2412_08059_amd import DeviceCSR
    return DeviceCSR.from_host(a, **kw)


def t64(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def band_ok(n_gpu, n_or):
    return abs(n_gpu - n_or) <= max(1, math.ceil(0.05 * n_or))


def _empty_rows_matrix():
    n = 300
    rng = np.random.default_rng(9)
    rows, cols, vals = [], [], []
    for i in range(n):
        if i % 7 == 3:
            continue   # empty row
        k = int(rng.integers(1, 12))
        c = np.unique(rng.integers(0, n, size=k))
        rows += [i] * len(c); cols += list(c); vals += list(rng.uniform(-2, 2, size=len(c)))
    return W.CSR.from_scipy(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)))


SPMV_CASES = {
    "poisson2d_64": lambda: W.poisson2d(64),
    "varcoef3d_20": lambda: W.varcoef3d(20, seed=1),
    "banded_20001": lambda: W.banded(20001, 8, seed=2),
    "er_30001": lambda: W.er_laplacian(30001, 16, seed=3),
    "star_5001_long_row": lambda: W.star(5001, mu=1.1),
    "empty_rows_300": _empty_rows_matrix,
    "one_by_one": lambda: W.CSR.from_scipy(sp.csr_matrix(np.array([[3.0]]))),
}


@pytest.mark.parametrize("name", list(SPMV_CASES))
@pytest.mark.parametrize("prec", [64, 32])
def test_spmv_bitwise(any_solver, torch_mod, name, prec):
    solver = any_solver
    a = SPMV_CASES[name]()
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, size=a.n)
    print(f"spmv case={name} n={a.n} nnz={a.nnz} prec={prec}", flush=True)
    A = dev(a, row_ptr_i64=(name == "banded_20001"))
    if prec == 64:
        st, y = solver.spmv(A, t64(torch_mod, x), 64)
        ref = oracle.spmv64(a, x)
        got = y.cpu().numpy()
    else:
        x32 = x.astype(np.float32)
        st, y = solver.spmv(A, torch_mod.from_numpy(x32).cuda(), 32)
        ref = oracle.spmv32(a, x32)
        got = y.cpu().numpy()
    assert st == 0
    assert np.array_equal(got.view(np.uint64 if prec == 64 else np.uint32),
                          ref.view(np.uint64 if prec == 64 else np.uint32))


BFS_CASES = [
    ("poisson2d_64", lambda: W.poisson2d(64), [0, 2080, 4095]),
    ("poisson3d_24", lambda: W.poisson3d(24), [0, 7000]),
    ("banded_100k", lambda: W.banded(100_000, 8, seed=0), [0, 50_000]),
    ("er_50k", lambda: W.er_laplacian(50_000, 16, seed=1), [0, 123]),
    ("xstar", lambda: W.extended_star(40, 25, extra_edges=30, seed=4), [0, 5]),
    ("path_3000", lambda: W.path(3000), [0, 1500]),
    # narrow bands (|i - j| <= 8): the one-workgroup kernel's bit-parallel levels
    ("band_holes_30001", lambda: __import__("workloads").paper_family.random_banded(30_001, 9, 0.4, 1.1, seed=3),
     [0, 15_000, 30_000]),
    ("path_1000", lambda: W.path(1000), [500]),
    ("banded_100003", lambda: W.banded(100_003, 8, seed=2), [100_002, 777]),
]


@pytest.mark.parametrize("name,gen,srcs", BFS_CASES, ids=[c[0] for c in BFS_CASES])
def test_bfs_distances_bitwise(bfs_solver, torch_mod, name, gen, srcs):
    solver = bfs_solver
    a = gen()
    A = dev(a)
    for s in srcs:
        print(f"bfs case={name} n={a.n} src={s}", flush=True)
        st, dist, ecc, far = solver.bfs(A, s)
        assert st == 0
        ref, recc = oracle.bfs(a, s)
        assert np.array_equal(dist.cpu().numpy(), ref)
        assert ecc == recc
        assert far == int(np.flatnonzero(ref == recc)[0])


def _union_graph():
    edges = [(i, i + 1) for i in range(199)] + [(200, j) for j in range(201, 260)]
    edges += [(300 + i, 300 + i + 1) for i in range(99)]
    ei = np.array([e[0] for e in edges]); ej = np.array([e[1] for e in edges])
    return W.generators._graph_matrix(420, ei, ej, 1.1, 1.0, "union")   # 400..419 isolated


PD_CASES = {
    "poisson2d_64": lambda: W.poisson2d(64),
    "poisson3d_20": lambda: W.poisson3d(20),
    "varcoef3d_16": lambda: W.varcoef3d(16, seed=2),
    "banded_100k": lambda: W.banded(100_000, 8, seed=0),
    "er_50k": lambda: W.er_laplacian(50_000, 16, seed=5),
    "xstar": lambda: W.extended_star(10, 30, extra_edges=20, seed=1),
    "union_components": _union_graph,
    "band_holes_30001": lambda: __import__("workloads").paper_family.random_banded(30_001, 9, 0.4, 1.1, seed=3),
    "diagonal_100": lambda: W.CSR.from_scipy(sp.identity(100, format="csr") * 2.0),
}


@pytest.mark.parametrize("name", list(PD_CASES))
def test_features_bitwise(bfs_solver, torch_mod, name):
    solver = bfs_solver
    a = PD_CASES[name]()
    _, b = W.rhs(a, seed=3)
    print(f"features case={name} n={a.n}", flush=True)
    st, f = solver.features(dev(a), t64(torch_mod, b), 20)
    assert st == 0
    assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == oracle.pseudo_diameter(a)
    assert (f.n, f.m) == (a.n, a.nnz)
    dummy = oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1]]), [2], k=1)
    r = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-10, model=dummy)
    assert f.k0_used == r.k0_used
    assert abs(f.v - r.v) <= 1e-9 * max(1.0, abs(r.v))


SOLVE_CASES = {
    "config1_poisson2d_64": (lambda: W.poisson2d(64), [1e-4, 1e-2, 1e-7]),
    "varcoef3d_24": (lambda: W.varcoef3d(24, seed=0), [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7]),
    "banded_30k": (lambda: W.banded(30_000, 8, seed=0), [1e-3, 1e-6]),
    "er_30k": (lambda: W.er_laplacian(30_000, 16, seed=0), [1e-3, 1e-5]),
    # offsets beyond 16 bits: 32-bit columns, the CG product in two launches
    "er_100k_wide": (lambda: W.er_laplacian(100_000, 16, seed=3), [1e-4, 1e-7]),
    "star_1001_absolute": (lambda: W.star(1001, mu=1.1), [1e-2, 1e-5]),
}


@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_solve_parity(any_solver, torch_mod, name):
    solver = any_solver
    gen, eps_list = SOLVE_CASES[name]
    a = gen()
    xs, b = W.rhs(a, seed=0)
    A = dev(a)
    B = t64(torch_mod, b)
    for e in [-1.0] + eps_list:
        print(f"solve case={name} n={a.n} eps1={e}", flush=True)
        st, x, s = solver.solve(A, B, e, 1e-10)
        r = oracle.solve(a, b, e, 1e-10)
        assert st == 0 and r.status == 0
        assert s.relres_final_true <= 1e-10
        assert band_ok(s.n1, r.n1), (s.n1, r.n1)
        assert band_ok(s.n2, r.n2), (s.n2, r.n2)
        xg = x.cpu().numpy()
        # the returned x meets eps2 on a residual recomputed by the oracle
        res = np.linalg.norm(b - oracle.spmv64(a, xg)) / np.linalg.norm(b)
        assert res <= 1e-10 * (1 + 1e-6)
        assert np.linalg.norm(xg - r.x) / np.linalg.norm(r.x) <= 1e-8


@pytest.mark.parametrize("eps1", [-1.0, 1e-5, 0.0])
def test_split_product_equals_fused_bitwise(torch_mod, eps1):
    """On a matrix with 32-bit columns the CG product runs as two launches
    (direction, then a one-vector gather); the arithmetic is the fused
    product's, so N1, N2, the eps1 class and x are the same bit for bit."""
    from paper_2412_08059_amd import Solver
    a = W.er_laplacian(100_000, 16, seed=3)
    _, b = W.rhs(a, seed=5)
    A, B = dev(a), t64(torch_mod, b)
    got = {}
    for split in ("1", "0"):
        s = Solver(a.n, a.nnz, model=TEST_MODEL, spmv_variant=2 if split == "1" else 1)
        st, x, S = s.solve(A, B, eps1, 1e-10)
        s.close()
        assert st == 0
        got[split] = (S.n1, S.n2, S.eps1_class, x.cpu().numpy().copy())
    print(f"eps1={eps1}: split n1/n2={got['1'][:2]} fused={got['0'][:2]}", flush=True)
    assert got["1"][:3] == got["0"][:3]
    assert np.array_equal(got["1"][3].view(np.uint64), got["0"][3].view(np.uint64))


def test_eps1_above_one_is_fp64_only_bitwise(solver, torch_mod):
    a = W.poisson2d(40)
    _, b = W.rhs(a, seed=1)
    A, B = dev(a), t64(torch_mod, b)
    st1, x1, s1 = solver.solve(A, B, 2.0, 1e-10)
    x1 = x1.cpu().numpy()
    st2, x2, s2 = solver.solve(A, B, -1.0, 1e-10)
    assert st1 == st2 == 0 and s1.n1 == 0 and s1.n2 == s2.n2
    assert np.array_equal(x1, x2.cpu().numpy())


def test_determinism_run_to_run(solver, torch_mod):
    a = W.varcoef3d(20, seed=4)
    _, b = W.rhs(a, seed=4)
    A, B = dev(a), t64(torch_mod, b)
    outs = []
    for _ in range(3):
        st, x, s = solver.solve(A, B, 1e-4, 1e-10)
        assert st == 0
        outs.append((x.cpu().numpy().copy(), s.n1, s.n2))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1:] == outs[0][1:]


AUTO_CASES = {
    "config1_poisson2d_64": lambda: W.poisson2d(64),
    "banded_20k": lambda: W.banded(20_000, 8, seed=7),
    "er_20k": lambda: W.er_laplacian(20_000, 16, seed=7),
    "varcoef3d_20": lambda: W.varcoef3d(20, seed=7),
}


@pytest.mark.parametrize("name", list(AUTO_CASES))
def test_algorithm2_auto_parity(solver, torch_mod, name):
    a = AUTO_CASES[name]()
    _, b = W.rhs(a, seed=7)
    model = oracle.load_model(TEST_MODEL)
    print(f"auto case={name} n={a.n}", flush=True)
    st, x, s = solver.solve(dev(a), t64(torch_mod, b), 0.0, 1e-10)
    r = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-10, model=model)
    assert st == 0 and r.status == 0
    f = s.feat
    assert (f.pdiam, f.bfs_t, f.bfs_u) == (r.ell, r.bfs_t, r.bfs_u)
    assert abs(f.v - r.v) <= 1e-9
    # the selector on the GPU's own features is bit-exact with the oracle's selector
    chi = [f.n, f.m, f.pdiam, f.v]
    t_or, _, _ = oracle.knn_select(model, chi)
    assert s.eps1_class == t_or
    assert s.eps1_class == r.eps1_class
    assert band_ok(s.n1, r.n1) and band_ok(s.n2, r.n2)
    assert s.relres_final_true <= 1e-10
    assert np.linalg.norm(x.cpu().numpy() - r.x) / np.linalg.norm(r.x) <= 1e-8


def test_select_eps1_bitwise_on_random_features(solver):
    from paper_2412_08059_amd import capi
    model = oracle.load_model(TEST_MODEL)
    rng = np.random.default_rng(0)
    lo, hi = model.fmin, model.fmax
    for i in range(300):
        chi = lo + (hi - lo) * rng.uniform(-0.1, 1.1, size=4)
        if i % 10 == 0:
            chi = model.feat[i % model.ns].copy()   # exact training sample -> zero distance
        f = capi.mpcg_features_t(int(round(chi[0])), int(round(chi[1])), int(round(chi[2])), 0, 0, 1, 20,
                                 float(chi[3]))
        q = [float(f.n), float(f.m), float(f.pdiam), f.v]
        st, e1, t = capi.mpcg_select_eps1(solver.ctx, f)
        assert st == 0
        t_or, _, _ = oracle.knn_select(model, q)
        assert t == t_or and e1 == [0, 0, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7][t]


# ------------------------------------------------------------ edge cases --

def test_edge_cases(solver, torch_mod):
    from paper_2412_08059_amd import capi, DeviceCSR
    # n = 1
    a = W.CSR.from_scipy(sp.csr_matrix(np.array([[4.0]])))
    st, x, s = solver.solve(dev(a), t64(torch_mod, [2.0]), 1e-4, 1e-10)
    assert st == 0 and abs(x.item() - 0.5) <= 1e-12
    # b = 0
    a = W.poisson2d(10)
    st, x, s = solver.solve(dev(a), t64(torch_mod, np.zeros(a.n)), 1e-4, 1e-10)
    assert st == 0 and s.n1 == 0 and s.n2 == 0 and not x.cpu().numpy().any()
    _, b = W.rhs(a, seed=0)
    B = t64(torch_mod, b)
    # malformed CSR
    bad = W.CSR(a.n, a.row_ptr.copy(), a.col.copy(), a.val.copy())
    bad.row_ptr[5], bad.row_ptr[6] = bad.row_ptr[6], bad.row_ptr[5]
    assert solver.solve(dev(bad), B, 1e-4, 1e-10)[0] == capi.MPCG_EINVAL
    bad = W.CSR(a.n, a.row_ptr.copy(), a.col.copy(), a.val.copy())
    bad.col[7] = a.n + 3
    assert solver.solve(dev(bad), B, 1e-4, 1e-10)[0] == capi.MPCG_EINVAL
    bad = W.CSR(a.n, a.row_ptr.copy(), a.col.copy(), a.val.copy())
    bad.col[a.row_ptr[4]], bad.col[a.row_ptr[4] + 1] = bad.col[a.row_ptr[4] + 1], bad.col[a.row_ptr[4]]
    assert solver.solve(dev(bad), B, 1e-4, 1e-10)[0] == capi.MPCG_EINVAL
    # bad tolerances
    assert solver.solve(dev(a), B, 1e-4, 0.0)[0] == capi.MPCG_EINVAL
    assert solver.solve(dev(a), B, -3.0, 1e-10)[0] == capi.MPCG_EINVAL
    # non-finite input
    bb = b.copy(); bb[3] = np.inf
    assert solver.solve(dev(a), t64(torch_mod, bb), 1e-4, 1e-10)[0] == capi.MPCG_ENONFINITE
    # not SPD: the FP32 phase breaks down and switches, the FP64 phase reports it
    neg = W.CSR.from_scipy(sp.csr_matrix(-np.eye(6)))
    st, x, s = solver.solve(dev(neg), t64(torch_mod, np.ones(6)), 1e-4, 1e-10)
    r = oracle.solve(neg, np.ones(6), 1e-4, 1e-10)
    assert st == capi.MPCG_ENOTSPD == r.status and (s.flags & capi.MPCG_FLAG_FP32_BREAKDOWN)


def test_iteration_caps_and_missing_model(torch_mod):
    from paper_2412_08059_amd import Solver, capi
    a = W.poisson2d(32)
    _, b = W.rhs(a, seed=0)
    s1 = Solver(a.n, a.nnz, maxit2=3, max_restarts=0)
    st, x, s = s1.solve(dev(a), t64(torch_mod, b), -1.0, 1e-10)
    r = oracle.solve(a, b, -1.0, 1e-10, maxit2=3, max_restarts=0)
    assert st == capi.MPCG_ENOCONV == r.status and s.n2 == r.n2 == 3
    st, x, s = s1.solve(dev(a), t64(torch_mod, b), 0.0, 1e-10)
    assert st == capi.MPCG_ENOMODEL
    s1.close()
    s2 = Solver(a.n, a.nnz, maxit1=2)
    st, x, s = s2.solve(dev(a), t64(torch_mod, b), 1e-7, 1e-10)
    assert st == 0 and s.n1 == 2 and (s.flags & capi.MPCG_FLAG_FP32_MAXIT)
    s2.close()
    s3 = Solver(10, 40)
    st, x, s = s3.solve(dev(a), t64(torch_mod, b), 1e-4, 1e-10)
    assert st == capi.MPCG_ENOMEM
    s3.close()
    # absolute tolerance mode (the Table 4 setting)
    star = W.star(1001, mu=1.1)
    xs = np.random.default_rng(0).uniform(1, 2, star.n)
    bs = star.to_scipy() @ xs
    s4 = Solver(star.n, star.nnz, tol_mode=1)
    for e in (1e-2, 1e-5, 1e-7):
        st, x, s = s4.solve(dev(star), t64(torch_mod, bs), e, 1e-10)
        r = oracle.solve(star, bs, e, 1e-10, tol_mode=1)
        assert st == 0 and (s.n1, s.n2) == (r.n1, r.n2)
    s4.close()


# ------------------------------------------------ full-size configurations --

def test_full_size_config2_3d_varcoef(solver, torch_mod):
    """128^3 variable-coefficient diffusion (the bench workload): bit-exact
    SpMV and pseudo-diameter at full size, and a solve whose residual the
    oracle recomputes."""
    a = W.varcoef3d(128, seed=0)
    xs, b = W.rhs(a, seed=0)
    A, B = dev(a), t64(torch_mod, b)
    print(f"full config2 n={a.n} nnz={a.nnz}", flush=True)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=a.n)
    st, y = solver.spmv(A, t64(torch_mod, x), 64)
    assert st == 0 and np.array_equal(y.cpu().numpy(), oracle.spmv64(a, x))
    x32 = x.astype(np.float32)
    st, y = solver.spmv(A, torch_mod.from_numpy(x32).cuda(), 32)
    assert st == 0 and np.array_equal(y.cpu().numpy(), oracle.spmv32(a, x32))
    st, f = solver.features(A, B, 20)
    assert st == 0 and (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == (381, a.n - 1, 0, 1)
    st, xg, s = solver.solve(A, B, 1e-4, 1e-10)
    assert st == 0 and s.relres_final_true <= 1e-10
    xg = xg.cpu().numpy()
    assert np.linalg.norm(b - oracle.spmv64(a, xg)) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-6)


@pytest.mark.parametrize("name", ["banded_1M", "er_1M"])
def test_full_size_config3_pseudo_diameter(solver, torch_mod, name):
    a = W.banded(1_000_000, 8, seed=0) if name == "banded_1M" else W.er_laplacian(1_000_000, 16, seed=0)
    _, b = W.rhs(a, seed=0)
    print(f"full config3 {name} n={a.n} nnz={a.nnz}", flush=True)
    st, f = solver.features(dev(a), t64(torch_mod, b), 20)
    assert st == 0
    ref = oracle.pseudo_diameter(a)
    assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == ref
    if name == "banded_1M":
        assert ref == (125_000, 999_993, 0, 1)


@pytest.mark.parametrize("name", ["config1_poisson2d_64", "varcoef3d_40"])
@pytest.mark.parametrize("t", [3, 4, 5, 6, 7])
def test_algorithm2_runahead_equals_algorithm1_bitwise(torch_mod, tmp_path, name, t):
    """With the class forced to t, Algorithm II (2BFS beside the FP32 phase,
    x~ copied at the first crossing of each candidate) must land on the state
    Algorithm I with eps1 = 10^-t stops in, whenever that stop is at or after
    the k0 = 20 prefix: same N1, N2 and the same x bit for bit."""
    from paper_2412_08059_amd import Solver
    a = W.poisson2d(64) if name.startswith("config1") else W.varcoef3d(40, seed=5)
    _, b = W.rhs(a, seed=11)
    mpath = tmp_path / f"one_class_{t}.txt"
    oracle.save_model(oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1], [2.0, 2, 2, 2]]), [t, t], k=1),
                      str(mpath))
    s = Solver(a.n, a.nnz, model=str(mpath))
    A, B = dev(a), t64(torch_mod, b)
    st2, x2, s2 = s.solve(A, B, 0.0, 1e-10)
    x2 = x2.cpu().numpy()
    st1, x1, s1 = s.solve(A, B, 10.0 ** -t, 1e-10)
    s.close()
    assert st1 == st2 == 0 and s2.eps1_class == t
    if s1.n1 >= 20:
        assert (s2.n1, s2.n2) == (s1.n1, s1.n2)
        assert np.array_equal(x2, x1.cpu().numpy())
    else:
        assert s2.n1 == 20   # the prefix already passed eps1; Algorithm II stops after it


@pytest.mark.parametrize("t", [7, 4])
def test_algorithm2_speculative_fp64_equals_algorithm1_bitwise(torch_mod, tmp_path, t):
    """A 2BFS far slower than the CG (tridiagonal band, mu = 1.1, n = 200000:
    2 x 199999 levels, while the FP32 recurrence passes 1e-7 within a few
    dozen iterations): the run-ahead crosses every candidate before the
    features are in, so the FP64 phase starts from the tightest candidate's
    state beside the BFS.  With the class forced to 7 that phase is kept, with
    4 it is discarded and the restart comes from the class-4 copy; both must
    equal Algorithm I with eps1 = 10^-t (N1, N2 and x bit for bit)."""
    from paper_2412_08059_amd import Solver
    from workloads import paper_family as PF
    a = PF.random_banded(200_000, 3, 1.0, 1.1, seed=4)
    _, b = W.rhs(a, seed=12)
    mpath = tmp_path / f"one_class_{t}.txt"
    oracle.save_model(oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1], [2.0, 2, 2, 2]]), [t, t], k=1),
                      str(mpath))
    s = Solver(a.n, a.nnz, model=str(mpath))
    A, B = dev(a), t64(torch_mod, b)
    st2, x2, s2 = s.solve(A, B, 0.0, 1e-10)
    x2 = x2.cpu().numpy()
    st1, x1, s1 = s.solve(A, B, 10.0 ** -t, 1e-10)
    s.close()
    print(f"class {t}: auto n1={s2.n1} n2={s2.n2} t_feat={s2.t_feat_ms:.1f} t_sp={s2.t_sp_ms:.1f} "
          f"t_dp={s2.t_dp_ms:.1f} ms; eps1 n1={s1.n1} n2={s1.n2}", flush=True)
    assert st1 == st2 == 0 and s2.eps1_class == t and s2.feat.pdiam == 199_999
    assert (s2.n1, s2.n2) == (s1.n1, s1.n2)
    assert np.array_equal(x2, x1.cpu().numpy())
    assert s2.relres_restart_true == s1.relres_restart_true
    # Whether the FP64 phase really began before the features were in
    # (t_sp_ms < t_feat_ms) depends on the main and side streams running on
    # different hardware queues, which a process with many live streams does
    # not guarantee; the result must be the same either way.


# ----------------------------------------------- Jacobi-preconditioned CG --

@pytest.fixture(scope="module")
def solver_jacobi(torch_mod):
    from paper_2412_08059_amd import Solver
    s = Solver(1_100_000, 12_000_000, model=TEST_MODEL, precond=1)
    yield s
    s.close()


# The x bar is 1e-8 except for the banded matrix: its condition number is
# 1.35e5 (shift 1e-4), two solves that both meet eps2 = 1e-10 may differ by up
# to 2 kappa eps2 = 2.7e-5, and the oracle's own unpreconditioned and Jacobi
# solutions of it differ by 1.2e-7; the GPU-oracle difference is held to 1e-7.
JACOBI_CASES = {
    "varcoef3d_24": (lambda: W.varcoef3d(24, seed=0), [1e-2, 1e-4, 1e-6], 1e-8),
    "banded_30k": (lambda: W.banded(30_000, 8, seed=0), [1e-3, 1e-6], 1e-7),
    "er_30k": (lambda: W.er_laplacian(30_000, 16, seed=0), [1e-3, 1e-5], 1e-8),
    "poisson2d_64": (lambda: W.poisson2d(64), [1e-4], 1e-8),
}


@pytest.mark.parametrize("name", list(JACOBI_CASES))
def test_jacobi_solve_parity(solver_jacobi, torch_mod, name):
    gen, eps_list, xtol = JACOBI_CASES[name]
    a = gen()
    _, b = W.rhs(a, seed=4)
    A, B = dev(a), t64(torch_mod, b)
    model = oracle.load_model(TEST_MODEL)
    for e in [-1.0] + eps_list + [0.0]:
        print(f"jacobi case={name} n={a.n} eps1={e}", flush=True)
        st, x, s = solver_jacobi.solve(A, B, e, 1e-10)
        r = oracle.solve(a, b, e, 1e-10, precond=1, model=model if e == 0.0 else None)
        assert st == 0 and r.status == 0
        assert s.relres_final_true <= 1e-10
        assert band_ok(s.n1, r.n1), (s.n1, r.n1)
        assert band_ok(s.n2, r.n2), (s.n2, r.n2)
        if e == 0.0:
            assert s.eps1_class == r.eps1_class
            assert abs(s.feat.v - r.v) <= 1e-9 * max(1.0, abs(r.v))
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - r.x) / np.linalg.norm(r.x) <= xtol


def test_jacobi_unit_diagonal_equals_cg_bitwise(solver, solver_jacobi, torch_mod):
    """M = I: the preconditioned kernels compute z = r / 1 = r and the same sums,
    so every bit equals the unpreconditioned solve."""
    n = 5000
    rng = np.random.default_rng(2)
    i = rng.integers(0, n, 4 * n); j = rng.integers(0, n, 4 * n)
    keep = i != j
    off = sp.coo_matrix((-rng.uniform(0, 0.1, keep.sum()), (i[keep], j[keep])), shape=(n, n)).tocsr()
    off = off + off.T
    off = off * (0.9 / np.asarray(abs(off).sum(axis=1)).ravel().max())
    a = W.CSR.from_scipy((off + sp.eye(n)).tocsr())
    _, b = W.rhs(a, seed=3)
    A, B = dev(a), t64(torch_mod, b)
    for e in (1e-3, 1e-6, -1.0):
        st0, x0, s0 = solver.solve(A, B, e, 1e-12)
        st1, x1, s1 = solver_jacobi.solve(A, B, e, 1e-12)
        assert st0 == 0 and st1 == 0
        assert (s0.n1, s0.n2) == (s1.n1, s1.n2)
        assert np.array_equal(x0.cpu().numpy().view(np.uint64), x1.cpu().numpy().view(np.uint64))


def test_jacobi_nonpositive_diagonal_is_not_spd(solver_jacobi, torch_mod):
    from paper_2412_08059_amd import capi
    a = W.poisson2d(16).to_scipy().tolil()
    a[7, 7] = -2.0
    m = W.CSR.from_scipy(sp.csr_matrix(a))
    st, _, s = solver_jacobi.solve(dev(m), t64(torch_mod, np.ones(m.n)), 1e-4, 1e-10)
    assert st == capi.MPCG_ENOTSPD


@pytest.mark.parametrize("t", [6, 7])
def test_algorithm2_runahead_beside_bfs_large_grid(torch_mod, tmp_path, t):
    """Above 8 x 256 slice groups (here 84^3 = 592,704 rows) the FP32 product
    takes one block per compute unit fewer while the 2BFS runs beside it, so
    its per-block partials of d.q group the rows differently from the full
    grid that Algorithm I uses: the two runs are the same method with another
    summation order, held to the parity band (per-phase counts within 5 %,
    x within 1e-8), not to bit equality."""
    from paper_2412_08059_amd import Solver
    a = W.varcoef3d(84, seed=2)
    _, b = W.rhs(a, seed=13)
    mpath = tmp_path / f"one_class_{t}.txt"
    oracle.save_model(oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1], [2.0, 2, 2, 2]]), [t, t], k=1),
                      str(mpath))
    s = Solver(a.n, a.nnz, model=str(mpath))
    A, B = dev(a), t64(torch_mod, b)
    st2, x2, s2 = s.solve(A, B, 0.0, 1e-10)
    x2 = x2.cpu().numpy()
    st1, x1, s1 = s.solve(A, B, 10.0 ** -t, 1e-10)
    x1 = x1.cpu().numpy()
    s.close()
    print(f"class {t}: auto n1={s2.n1} n2={s2.n2}; eps1 n1={s1.n1} n2={s1.n2}; "
          f"bitwise={np.array_equal(x1, x2)}", flush=True)
    assert st1 == st2 == 0 and s2.eps1_class == t
    assert s1.relres_final_true <= 1e-10 and s2.relres_final_true <= 1e-10
    assert band_ok(s2.n1, s1.n1) and band_ok(s2.n2, s1.n2)
    assert np.linalg.norm(x2 - x1) / np.linalg.norm(x1) <= 1e-8
