"""The 2BFS on bit vectors over the diagonals against the oracle's BFS.

When every stored entry lies on one of at most 16 diagonals (grids, bands),
the library can form each BFS level from bit vectors of all rows instead of a
queue.  Distances are unique, so the bar is bit-exact: distances, eccentricity
and farthest vertex of a sweep, and the 2BFS features (section on the matrix
graph diameter) equal the oracle's.  The cases span the word and wave edges
(n not a multiple of 32 or 64), the most diagonals the path takes (16) and more
(18: the queue kernels take over), holes in the diagonals, a disconnected
pattern (first sweep on diagonals, then the component path) and a pattern
with the main diagonal only.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


DIA_TUNINGS = {"tiles": {"bfs_dia": 2, "bfs_dia_tiles": 1, "bfs_persist": 0},
               "levels": {"bfs_dia": 2, "bfs_dia_tiles": 0, "bfs_persist": 0},
               "levels_persist": {"bfs_dia": 2, "bfs_dia_tiles": 0, "bfs_persist": 1}}


@pytest.fixture(scope="module", params=list(DIA_TUNINGS))
def dia_solver(request, torch_mod):
    """Several levels per launch (temporal tiles where a tile holds 8 or more
    levels, else two levels per launch), or one launch per level; with
    bfs_persist the sweeps that the diagonals cannot take (a pattern that is
    not connected) run on the persistent queue kernel."""
    from paper_2412_08059_amd import Solver
    s = Solver(2_200_000, 20_000_000, tuning=DIA_TUNINGS[request.param])
    s.dia_tuning = DIA_TUNINGS[request.param]
    yield s
    s.close()


def dev(a):
    from paper_2412_08059_amd import DeviceCSR
    return DeviceCSR.from_host(a)


def _diagonals(n, offsets, keep=1.0, seed=0):
    """Symmetric pattern on +-offsets (each entry kept with probability
    `keep`, mirrored), diagonally dominant values."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for d in offsets:
        i = np.arange(n - d)
        m = rng.random(n - d) < keep
        rows += [i[m], i[m] + d]
        cols += [i[m] + d, i[m]]
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    off = sp.csr_matrix((-np.ones(len(r)), (r, c)), shape=(n, n))
    deg = np.asarray(abs(off).sum(axis=1)).ravel()
    return W.CSR.from_scipy((off + sp.diags(deg + 1.0)).tocsr())


CASES = {
    "poisson2d_61": lambda: W.poisson2d(61),                      # n = 3721, ragged word and wave
    "poisson3d_33": lambda: W.poisson3d(33),                      # 6 diagonals, n = 35937
    "varcoef3d_40": lambda: W.varcoef3d(40, seed=4),
    "banded_70001_16diag": lambda: W.banded(70_001, 8, seed=1),   # +-1..+-8: 16 diagonals
    "banded_5001_18diag": lambda: _diagonals(5001, list(range(1, 9)) + [40]),   # 18: queue path
    "holes_100003": lambda: _diagonals(100_003, [1, 3, 130, 4000], keep=0.7, seed=2),
    "wide_offsets_40000": lambda: _diagonals(40_000, [1, 9999, 20000], seed=3),
    "two_components": lambda: _diagonals(3000, [2]),              # even and odd rows
    "path_65": lambda: W.path(65),
    # beyond one tile's 8192 words with short diagonals: several levels per
    # launch over several tiles (the "tiles" tuning)
    "poisson2d_700": lambda: W.poisson2d(700),
    "grid3d_40x40x200": lambda: _diagonals(320_000, [1, 40, 1600], seed=4),
    "holes_600001": lambda: _diagonals(600_001, [1, 3, 130, 4000], keep=0.7, seed=5),
    # halo of 256 words per level (8 levels per launch) and of 257 (one launch per level)
    "reach_256_400000": lambda: _diagonals(400_000, [1, 8160], seed=6),
    "reach_257_400000": lambda: _diagonals(400_000, [1, 8192], seed=7),
    "diagonal_only_97": lambda: W.CSR.from_scipy(sp.identity(97, format="csr") * 3.0),
}


def _oracle_sweep(a, s):
    ref, ecc = oracle.bfs(a, s)
    return ref, ecc, int(np.flatnonzero(ref == ecc)[0])


@pytest.mark.parametrize("name", list(CASES))
def test_dia_sweeps_bitwise(dia_solver, torch_mod, name):
    a = CASES[name]()
    A = dev(a)
    rng = np.random.default_rng(11)
    srcs = sorted({0, a.n - 1, int(rng.integers(0, a.n))})
    for s in srcs:
        print(f"dia bfs case={name} n={a.n} src={s}", flush=True)
        st, dist, ecc, far = dia_solver.bfs(A, s)
        assert st == 0
        ref, recc, rfar = _oracle_sweep(a, s)
        assert np.array_equal(dist.cpu().numpy(), ref)
        assert (ecc, far) == (recc, rfar)


@pytest.mark.parametrize("name", list(CASES))
def test_dia_features_bitwise(dia_solver, torch_mod, name):
    a = CASES[name]()
    _, b = W.rhs(a, seed=5)
    print(f"dia features case={name} n={a.n}", flush=True)
    st, f = dia_solver.features(dev(a), torch_mod.from_numpy(b).cuda(), 20)
    assert st == 0
    assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == oracle.pseudo_diameter(a)


def test_dia_grid_size_of_the_solve_workload(dia_solver, torch_mod):
    """The 3-D variable-coefficient 128^3 grid (2,097,152 rows, 7 diagonals)
    through Algorithm II: the 2BFS ran on diagonals (flag set) and gave the
    oracle's features; with bfs_dia = 0 the queue kernels give the same."""
    a = W.varcoef3d(128, seed=0)
    _, b = W.rhs(a, seed=0)
    A = dev(a)
    B = torch_mod.from_numpy(b).cuda()
    ref = oracle.pseudo_diameter(a)
    print("dia features 128^3", flush=True)
    st, f = dia_solver.features(A, B, 20)
    assert st == 0 and (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == ref
    dia_solver.set_tuning({"bfs_dia": 0, "bfs_persist": 0})
    try:
        st, g = dia_solver.features(A, B, 20)
        assert st == 0 and (g.pdiam, g.bfs_t, g.bfs_u, g.n_components) == ref
    finally:
        dia_solver.set_tuning(dia_solver.dia_tuning)
    assert ref[0] == 3 * 127


def test_dia_flag_in_algorithm2(torch_mod):
    """The solve reports MPCG_FLAG_BFS_DIA when its 2BFS ran on diagonals,
    and not when the tuning turns that off."""
    import os
    from paper_2412_08059_amd import Solver, capi
    model = os.path.join(os.path.dirname(__file__), "golden", "knn_model_test.txt")
    a = W.poisson3d(48)
    _, b = W.rhs(a, seed=1)
    A = dev(a)
    B = torch_mod.from_numpy(b).cuda()
    for mode, tiles, want in ((2, 0, True), (1, 0, True), (1, 1, True), (0, 0, False)):
        s = Solver(a.n, a.nnz, model=model, tuning={"bfs_dia": mode, "bfs_dia_tiles": tiles})
        try:
            print(f"dia flag mode={mode} tiles={tiles}", flush=True)
            st, x, stats = s.solve(A, B, 0.0, 1e-10)
            assert st == 0 and stats.relres_final_true <= 1e-10
            assert bool(stats.flags & capi.MPCG_FLAG_BFS_DIA) == want
            assert (stats.feat.pdiam, stats.feat.bfs_t, stats.feat.bfs_u) == oracle.pseudo_diameter(a)[:3]
        finally:
            s.close()
