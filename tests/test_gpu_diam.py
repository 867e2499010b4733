"""GPU parity of mpcg_diameter_multi (multi-start 2BFS and the effective
diameter) against the oracle: every output bit-exact (integer work), on
graphs that exercise the one-workgroup kernel and its window (bands, paths),
the multi-block level kernel (grids, random graphs), disconnected graphs
with isolated vertices, and the error paths."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from workloads import paper_family as PF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2412_08059_amd import Solver
    s = Solver(300_000, 3_000_000)
    yield s
    s.close()


def _union():
    return W.CSR.from_scipy(sp.block_diag([W.path(300).to_scipy(), W.poisson2d(30).to_scipy(),
                                           sp.csr_matrix(np.array([[2.0]]))]).tocsr())


CASES = {
    "grid2d_60": lambda: W.poisson2d(60),
    "varcoef3d_40": lambda: W.varcoef3d(40, seed=1),
    "band_20k": lambda: W.banded(20_000, 8, seed=2),
    "path_5000": lambda: W.path(5000),
    "er_20k": lambda: W.er_laplacian(20_000, 16, seed=3),
    "xstar": lambda: PF.perturbed_extended_star(25, 40, 1.1, seed=4),
    "random_1000": lambda: PF.random_sparse(1000, 1.0, 3.0, seed=5),
    "band_sparse": lambda: PF.random_banded(1000, 9, 0.4, 1.1, seed=6),
    "union": _union,
}


@pytest.mark.parametrize("name", list(CASES))
def test_diameter_multi_bitwise(solver, name):
    from paper_2412_08059_amd import DeviceCSR
    a = CASES[name]()
    rng = np.random.default_rng(len(name))
    starts = sorted(set(rng.integers(0, a.n, size=6).tolist()) | {a.n - 1})
    A = DeviceCSR.from_host(a)
    for q in (0.5, 0.9, 1.0):
        print(f"diameter_multi case={name} n={a.n} starts={starts} q={q}", flush=True)
        st, d = solver.diameter_multi(A, starts, q)
        assert st == 0
        want = oracle.diameter_multi(a, starts, q)
        assert (d.pdiam, d.pdiam_multi, d.eff_diam, d.pairs, d.best_start) == want


def test_diameter_multi_errors(solver):
    from paper_2412_08059_amd import DeviceCSR, capi
    a = W.poisson2d(10)
    A = DeviceCSR.from_host(a)
    assert solver.diameter_multi(A, [100], 0.9)[0] == capi.MPCG_EINVAL
    assert solver.diameter_multi(A, [-1], 0.9)[0] == capi.MPCG_EINVAL
    assert solver.diameter_multi(A, [0], 0.0)[0] == capi.MPCG_EINVAL
    assert solver.diameter_multi(A, [0], 1.5)[0] == capi.MPCG_EINVAL
    st, d = solver.diameter_multi(A, [], 0.9)
    assert st == 0 and (d.pdiam_multi, d.eff_diam, d.pairs, d.best_start) == (d.pdiam, 0, 0, -1)
