"""GPU parity of the two-stage Jacobi method (mpcg_solve_jacobi) against the
oracle.  Every row is the same arithmetic on both sides (the off-diagonal
fma chain in stored order, one fma for the residual, one division), so the
iterates are bitwise equal; only the order of the ||r||^2 sum differs, which
can move a stop by one update.  Bars: N1 and N2 within 1 of the oracle's;
when both are equal, x bitwise equal to the oracle's; final FP64 residual
<= eps2; the FP32 cap flag as the oracle's."""

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
    s = Solver(1_100_000, 24_000_000)
    yield s
    s.close()


CASES = {
    "star_1001": (lambda: W.star(1001, mu=1.1), "u12"),
    "path_1001": (lambda: W.path(1001, mu=1.1), "u12"),
    "xstar": (lambda: PF.perturbed_extended_star(20, 50, 3.0, seed=1), "u12"),
    "random_mu3": (lambda: PF.random_sparse(5000, 2.0, 3.0, seed=2), "u12"),
    "banded_mu1.1": (lambda: PF.random_banded(4000, 21, 0.6, 1.1, seed=3), "u12"),
    "random_1M_mu3": (lambda: PF.random_sparse(1_000_000, 1.0, 3.0, seed=4), "u12"),
    "grid_shifted": (lambda: W.CSR.from_scipy((W.poisson2d(300).to_scipy() + sp.identity(90000) * 4.0).tocsr()),
                     "pm1"),
}


def _rhs(a, how, seed):
    if how == "u12":
        return PF.paper_rhs(a, seed)[1]
    return W.rhs(a, seed=seed)[1]


@pytest.mark.parametrize("name", list(CASES))
def test_jacobi_two_stage_matches_oracle(solver, name):
    import torch
    from paper_2412_08059_amd import DeviceCSR, capi
    gen, how = CASES[name]
    a = gen()
    b = _rhs(a, how, 11)
    A = DeviceCSR.from_host(a)
    B = torch.from_numpy(b).cuda()
    for e in (1e-2, 1e-4, 1e-6, 1e-7, -1.0):
        print(f"jacobi case={name} n={a.n} eps1={e}", flush=True)
        st, x, s = solver.solve_jacobi(A, B, e, 1e-10)
        r = oracle.solve_jacobi(a, b, e, 1e-10)
        assert st == r.status == 0, (st, r.status)
        assert s.relres_final_true <= 1e-10
        assert abs(s.n1 - r.n1) <= 1 and abs(s.n2 - r.n2) <= 1, (e, s.n1, r.n1, s.n2, r.n2)
        assert (s.flags & capi.MPCG_FLAG_FP32_MAXIT) == (r.flags & oracle.FLAG_FP32_MAXIT)
        if (s.n1, s.n2) == (r.n1, r.n2):
            assert np.array_equal(x.cpu().numpy().view(np.uint64), r.x.view(np.uint64)), e


def test_jacobi_errors(solver):
    import torch
    from paper_2412_08059_amd import DeviceCSR, capi
    m = W.poisson2d(8).to_scipy().tolil()
    m[5, 5] = -2.0
    a = W.CSR.from_scipy(sp.csr_matrix(m))
    A = DeviceCSR.from_host(a)
    B = torch.ones(a.n, dtype=torch.float64, device="cuda")
    assert solver.solve_jacobi(A, B, 1e-4, 1e-10)[0] == capi.MPCG_ENOTSPD
    good = DeviceCSR.from_host(W.poisson2d(8))
    assert solver.solve_jacobi(good, B, 0.0, 1e-10)[0] == capi.MPCG_EINVAL      # no kNN eps1 here
    assert solver.solve_jacobi(good, B, 1e-4, -1.0)[0] == capi.MPCG_EINVAL
    Z = torch.zeros(64, dtype=torch.float64, device="cuda")
    st, x, s = solver.solve_jacobi(good, Z, 1e-4, 1e-10)
    assert st == 0 and s.n1 == 0 and s.n2 == 0 and torch.all(x == 0)
