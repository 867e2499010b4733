"""Pins of the oracle's Jacobi-preconditioned stages (the "CG with
preconditioning" procedure with M = diag(A)) against facts that do not come
from the oracle itself."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads as W


def _unit_diag_matrix(n=400, seed=3):
    """SPD, diagonal exactly 1.0 (strictly diagonally dominant graph matrix)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, 3 * n)
    j = rng.integers(0, n, 3 * n)
    keep = i != j
    off = sp.coo_matrix((-rng.uniform(0.0, 0.1, keep.sum()), (i[keep], j[keep])), shape=(n, n)).tocsr()
    off = off + off.T
    rows = np.asarray(abs(off).sum(axis=1)).ravel()
    scale = 0.9 / max(rows.max(), 1e-300)
    a = (off * scale + sp.eye(n)).tocsr()
    a.sum_duplicates()
    a.sort_indices()
    assert np.all(a.diagonal() == 1.0)
    return W.CSR.from_scipy(a)


@pytest.mark.parametrize("eps1", [1e-3, 1e-6, -1.0])
def test_unit_diagonal_reduces_to_cg_bitwise(eps1):
    """M = I: z = r / 1 = r exactly, so every stage is the unpreconditioned CG."""
    a = _unit_diag_matrix()
    _, b = W.rhs(a, seed=1)
    r0 = oracle.solve(a, b, eps1, 1e-12)
    r1 = oracle.solve(a, b, eps1, 1e-12, precond=1)
    assert r0.status == 0 and r1.status == 0
    assert (r0.n1, r0.n2) == (r1.n1, r1.n2)
    assert np.array_equal(r0.x.view(np.uint64), r1.x.view(np.uint64))


def test_unit_diagonal_auto_reduces_to_cg_bitwise():
    a = _unit_diag_matrix(seed=5)
    _, b = W.rhs(a, seed=2)
    model = oracle.KnnModel.from_samples(np.array([[400.0, 3000, 8, 0.5], [500.0, 4000, 12, 0.8]]), [4, 6], k=1)
    r0 = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-12, model=model)
    r1 = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-12, model=model, precond=1)
    assert (r0.n1, r0.n2, r0.eps1_class, r0.v) == (r1.n1, r1.n2, r1.eps1_class, r1.v)
    assert np.array_equal(r0.x.view(np.uint64), r1.x.view(np.uint64))


def test_diagonal_matrix_one_iteration():
    """A diagonal: M^-1 b is the solution, so the FP64 stage stops after one step."""
    n = 300
    rng = np.random.default_rng(0)
    dvals = rng.uniform(0.5, 50.0, n)
    a = W.CSR.from_scipy(sp.diags(dvals).tocsr())
    b = rng.uniform(-1, 1, n)
    r = oracle.solve(a, b, -1.0, 1e-13, precond=1)
    assert r.status == 0 and r.n2 == 1
    assert np.allclose(r.x, b / dvals, rtol=1e-14, atol=0)


def test_dense_spd_matches_direct_solve():
    for seed in range(4):
        A, a = W.random_spd_dense(24, seed=seed)
        rng = np.random.default_rng(seed)
        b = rng.uniform(-1, 1, 24)
        r = oracle.solve(a, b, -1.0, 1e-12, precond=1)
        xs = np.linalg.solve(A, b)
        kappa = np.linalg.cond(A)
        assert r.status == 0
        assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 10 * kappa * 1e-12


@pytest.mark.parametrize("gen", [lambda: W.varcoef3d(10, seed=2), lambda: W.banded(3000, 8, seed=1),
                                 lambda: W.er_laplacian(2000, 16, seed=4)])
def test_fp64_stage_iterations_match_scipy_pcg(gen):
    """scipy's preconditioned cg (M^-1 = diag(A)^-1, stop on ||r|| <= rtol ||b||,
    x0 = 0) is an independent implementation of the same recurrence."""
    a = gen()
    _, b = W.rhs(a, seed=0)
    A = a.to_scipy()
    dinv = 1.0 / A.diagonal()
    M = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    count = [0]
    spla.cg(A, b, rtol=1e-10, atol=0.0, maxiter=100000, M=M, callback=lambda xk: count.__setitem__(0, count[0] + 1))
    r = oracle.solve(a, b, -1.0, 1e-10, precond=1)
    assert r.status == 0
    assert abs(r.n2 - count[0]) <= 2, (r.n2, count[0])


def test_jacobi_helps_badly_scaled_system():
    """Diagonal scaling removes the coefficient spread of the variable-coefficient
    problem (three decades): far fewer FP64 iterations, same solution."""
    a = W.varcoef3d(14, seed=1, decades=3)
    xs, b = W.rhs(a, seed=1)
    r0 = oracle.solve(a, b, -1.0, 1e-10)
    r1 = oracle.solve(a, b, -1.0, 1e-10, precond=1)
    assert r0.status == 0 and r1.status == 0
    assert r1.n2 < 0.7 * r0.n2
    assert np.linalg.norm(r1.x - r0.x) / np.linalg.norm(r0.x) <= 1e-7


def test_two_stage_jacobi_properties():
    a = W.varcoef3d(12, seed=3)
    _, b = W.rhs(a, seed=3)
    n1 = []
    for e in (1e-2, 1e-4, 1e-6):
        r = oracle.solve(a, b, e, 1e-10, precond=1)
        assert r.status == 0 and r.relres_final_true <= 1e-10
        n1.append(r.n1)
    assert n1 == sorted(n1)
    r2 = oracle.solve(a, b, 2.0, 1e-10, precond=1)
    rd = oracle.solve(a, b, -1.0, 1e-10, precond=1)
    assert r2.n1 == 0 and np.array_equal(r2.x.view(np.uint64), rd.x.view(np.uint64))


def test_missing_or_nonpositive_diagonal_is_not_spd():
    a = W.poisson2d(6).to_scipy().tolil()
    a[3, 3] = 0.0
    m = sp.csr_matrix(a)
    m.eliminate_zeros()
    b = np.ones(36)
    assert oracle.solve(W.CSR.from_scipy(m), b, 1e-4, 1e-10, precond=1).status == oracle.ENOTSPD
    a = W.poisson2d(6).to_scipy().tolil()
    a[5, 5] = -1.0
    assert oracle.solve(W.CSR.from_scipy(sp.csr_matrix(a)), b, 1e-4, 1e-10, precond=1).status == oracle.ENOTSPD
