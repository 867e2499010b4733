"""Pins of the oracle's two-stage Jacobi method (the section on rounding-error
growth in other iterative methods) against facts that do not come from it:
  * error propagation e_k = T^k e_0, T = D^{-1}(L + U) applied with the sign
    that solves A x = b (dense matrix powers, numpy);
  * a diagonal matrix is solved by one update;
  * eps1 >= 1 leaves the FP32 stage at once: bitwise the FP64-only solve;
  * the FP32 stage of a looser eps1 is a prefix of a tighter one (same
    iterates): N1 is monotone and the FP64 stage starts from the same x~;
  * the iteration count obeys the contraction bound of a strictly
    diagonally dominant matrix, ||T||_inf <= 1/mu;
  * the table's qualitative finding: on the path graph (mu = 1.1) FP32
    rounding stops the residual short of 1e-7 (the stage hits its cap).
The paper's Jacobi table counts themselves are parity unpinned: with the
stated mu = 1.1 the contraction factor of both graphs is 1/1.1 per iteration,
which needs ~240 FP64 iterations to 1e-10, far more than the printed ones."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from workloads import paper_family as PF


def _dd(n=30, seed=0, mu=2.0):
    a = PF.random_sparse(n, 1.0, mu, seed=seed)
    return a


@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_error_propagation_matches_matrix_powers(k):
    a = _dd(seed=1)
    A = a.to_scipy().toarray()
    rng = np.random.default_rng(2)
    xs = rng.uniform(1, 2, a.n)
    b = A @ xs
    xstar = np.linalg.solve(A, b)
    D = np.diag(np.diag(A))
    T = -np.linalg.solve(D, A - D)           # D^{-1}(b - (L+U)x) = T x + D^{-1} b
    e = np.linalg.matrix_power(T, k) @ (np.zeros(a.n) - xstar)
    r = oracle.solve_jacobi(a, b, -1.0, 1e-300, maxit2=k)
    assert r.status == oracle.ENOCONV and r.n2 == k
    assert np.linalg.norm(r.x - (xstar + e)) <= 1e-12 * np.linalg.norm(xstar)


def test_diagonal_matrix_one_update():
    rng = np.random.default_rng(0)
    dv = rng.uniform(0.5, 20.0, 200)
    a = W.CSR.from_scipy(sp.diags(dv).tocsr())
    b = rng.uniform(-1, 1, 200)
    r = oracle.solve_jacobi(a, b, -1.0, 1e-13)
    assert r.status == 0 and r.n2 == 1
    assert np.allclose(r.x, b / dv, rtol=1e-15, atol=0)


def test_eps1_above_one_is_fp64_only_bitwise():
    a = _dd(200, seed=3, mu=3.0)
    _, b = PF.paper_rhs(a, 3)
    r0 = oracle.solve_jacobi(a, b, -1.0, 1e-10)
    r1 = oracle.solve_jacobi(a, b, 2.0, 1e-10)
    assert r1.n1 == 0 and r1.n2 == r0.n2
    assert np.array_equal(r0.x.view(np.uint64), r1.x.view(np.uint64))


def test_fp32_stage_is_a_prefix():
    a = PF.random_banded(500, 9, 0.8, 3.0, seed=5)
    _, b = PF.paper_rhs(a, 5)
    n1 = [oracle.solve_jacobi(a, b, e, 1e-10).n1 for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]
    assert n1 == sorted(n1) and n1[0] < n1[-1]
    # stopping the tight run at the loose run's N1 gives the same x~, so the
    # same FP64 stage
    loose = oracle.solve_jacobi(a, b, 1e-3, 1e-10)
    capped = oracle.solve_jacobi(a, b, 1e-30, 1e-10, maxit1=loose.n1)
    assert capped.n1 == loose.n1 and capped.n2 == loose.n2
    assert np.array_equal(capped.x.view(np.uint64), loose.x.view(np.uint64))


@pytest.mark.parametrize("mu", [1.5, 3.0, 10.0])
def test_contraction_bound(mu):
    """||e_k||_inf <= mu^-k ||e_0||_inf and ||r_k|| <= ||A||_2 ||e_k||_2, so
    the FP64 count to eps2 is at most the k at which
    ||A||_2 sqrt(n) mu^-k ||x*||_inf <= eps2 ||b||."""
    a = PF.random_sparse(300, 2.0, mu, seed=7)
    A = a.to_scipy().toarray()
    xs = np.random.default_rng(7).uniform(1, 2, a.n)
    b = A @ xs
    r = oracle.solve_jacobi(a, b, -1.0, 1e-10)
    assert r.status == 0
    an = np.linalg.norm(A, 2)
    kmax = math.ceil(math.log(an * math.sqrt(a.n) * np.abs(xs).max() / (1e-10 * np.linalg.norm(b))) / math.log(mu))
    assert r.n2 <= kmax


def test_path_fp32_cannot_reach_1e7():
    a = W.path(1001, mu=1.1)
    rng = np.random.default_rng(0)
    b = a.to_scipy() @ rng.uniform(1, 2, a.n)
    r = oracle.solve_jacobi(a, b, 1e-7, 1e-10)
    assert r.status == 0 and (r.flags & oracle.FLAG_FP32_MAXIT) and r.relres_sp > 1e-7
    r5 = oracle.solve_jacobi(a, b, 1e-5, 1e-10)
    assert not (r5.flags & oracle.FLAG_FP32_MAXIT)


def test_errors():
    a = W.poisson2d(5).to_scipy().tolil()
    a[3, 3] = -1.0
    b = np.ones(25)
    assert oracle.solve_jacobi(W.CSR.from_scipy(sp.csr_matrix(a)), b, 1e-4, 1e-10).status == oracle.ENOTSPD
    bb = b.copy()
    bb[4] = np.nan
    assert oracle.solve_jacobi(W.poisson2d(5), bb, 1e-4, 1e-10).status == oracle.ENONFINITE
