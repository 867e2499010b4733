"""Pins of the oracle's final-check restart, its initial guess x0, the
FP32-accumulated dot products (dot_acc = 1), the CG-Lanczos condition
estimate and the multi-threaded row loops (no GPU).

The final check follows the loop test of the CG procedure in the paper's
"Conjugate Gradient Method" section, applied to the true residual b - A x
(Algorithm I returns x only once that test passes): when it fails, CG starts
again from x with r = b - A x.  So a solve that restarts once must equal, bit
for bit, the FP64-only CG that starts from the pre-restart iterate."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

# A band with a weak diagonal shift and a smooth solution: the recursive
# residual falls below eps2 = 3e-12 while the true residual is still several
# times larger, so the final check fails once and the restart then passes.
RESTART_EPS2 = 3e-12


@pytest.fixture(scope="module")
def restart_case():
    a = W.banded(20000, 8, seed=1, shift=1e-4)
    xs, b = W.smooth_rhs(a)
    return a, xs, b


@pytest.mark.parametrize("eps1", [oracle.EPS1_NONE, 1e-4])
def test_final_restart_equals_fp64_cg_from_the_pre_restart_iterate(restart_case, eps1):
    a, xs, b = restart_case
    pre = oracle.solve(a, b, eps1, RESTART_EPS2, max_restarts=0)
    assert pre.status == oracle.ENOCONV and pre.restarts == 0
    assert pre.relres_final_true > 2 * RESTART_EPS2          # the check fails clearly
    full = oracle.solve(a, b, eps1, RESTART_EPS2)
    assert full.status == oracle.OK
    assert full.restarts == 1 and full.flags & oracle.FLAG_FINAL_RESTARTED
    assert full.relres_final_true <= RESTART_EPS2
    post = oracle.solve(a, b, oracle.EPS1_NONE, RESTART_EPS2, x0=pre.x, max_restarts=0)
    assert post.status == oracle.OK and post.restarts == 0
    assert np.array_equal(full.x, post.x)
    assert full.n2 == pre.n2 + post.n2
    assert full.n1 == pre.n1
    assert full.relres_final_true == post.relres_final_true
    # the restart's residual is the true residual of the pre-restart iterate
    assert post.relres_restart_true == pre.relres_final_true


def test_x0_exact_solution_takes_no_iteration():
    a = W.poisson2d(16)
    x = np.random.default_rng(5).integers(-50, 50, size=a.n).astype(np.float64)
    b = a.to_scipy() @ x                    # integer data: b = A x exactly
    r = oracle.solve(a, b, oracle.EPS1_NONE, 1e-12, x0=x)
    assert r.status == oracle.OK and r.n2 == 0 and r.relres_restart_true == 0.0
    assert np.array_equal(r.x, x)
    # the FP32 stage starts from float32(x0) (exact here) with r~ = b~ - A~ x~0 = 0
    r32 = oracle.solve(a, b, 1e-4, 1e-12, x0=x)
    assert r32.n1 == 0 and r32.n2 == 0 and np.array_equal(r32.x, x)


def test_x0_zero_is_the_default():
    a = W.poisson2d(24)
    _, b = W.rhs(a, seed=3)
    for e1 in (oracle.EPS1_NONE, 1e-5):
        r0 = oracle.solve(a, b, e1, 1e-10)
        rz = oracle.solve(a, b, e1, 1e-10, x0=np.zeros(a.n))
        assert (r0.n1, r0.n2) == (rz.n1, rz.n2) and np.array_equal(r0.x, rz.x)


# ------------------------------------------------------ dot_acc = 1 (FP32) --

@pytest.mark.parametrize("p", [-2, 3])
def test_fp32_dots_on_scaled_identity_are_one_exact_step(p):
    """On 2^p I, delta = d.(2^p d) is 2^p times gamma = r.r in either
    accumulation (scaling by a power of two is exact at every step of the
    chain), so alpha = 2^-p exactly and x~ = b~ / 2^p after one iteration."""
    n = 50
    a = W.CSR.from_scipy(2.0 ** p * np.eye(n))
    b = np.random.default_rng(7).uniform(-1, 1, n)
    b32 = b.astype(np.float32).astype(np.float64)
    for acc in (0, 1):
        # eps2 above ||b - b~|| / ||b|| (~6e-8): the FP64 stage takes no step
        r = oracle.solve(a, b, 1e-3, 1e-6, dot_acc=acc)
        assert r.n1 == 1 and r.relres_sp == 0.0 and r.n2 == 0
        assert np.array_equal(r.x, b32 / 2.0 ** p)


def test_fp32_dot_accumulation_precision():
    """With eps1 above 1 the FP32 stage stops at once and relres_sp is
    sqrt(b~.b~) / ||b||: within n u64 of the exact value when the products are
    summed in FP64, and off by far more than that (but within n u32) when the
    sum is an FP32 chain."""
    n = 3000
    b = np.random.default_rng(11).uniform(0.5, 1.5, n)
    a = W.CSR.from_scipy(np.eye(n))
    b32 = b.astype(np.float32)
    exact = sum(Fraction(float(v)) ** 2 for v in b32)
    bb = sum(Fraction(float(v)) ** 2 for v in b)
    ref = math.sqrt(exact) / math.sqrt(bb)
    r64 = oracle.solve(a, b, 2.0, 1e-10, dot_acc=0)
    r32 = oracle.solve(a, b, 2.0, 1e-10, dot_acc=1)
    e64 = abs(r64.relres_sp - ref) / ref
    e32 = abs(r32.relres_sp - ref) / ref
    assert e64 <= n * 2.0 ** -53
    assert e32 <= n * 2.0 ** -24
    assert e32 > 1e3 * max(e64, 2.0 ** -53)


def test_fp32_dots_keep_the_prefix_property_and_reach_eps2():
    a = W.poisson2d(48)
    _, b = W.rhs(a, seed=0)
    n1s = []
    for e in oracle.cost.EPS1_CANDIDATES:
        r = oracle.solve(a, b, e, 1e-10, dot_acc=1)
        assert r.status == oracle.OK and r.relres_final_true <= 1e-10
        r7 = oracle.solve(a, b, 1e-7, 1e-10, dot_acc=1, maxit1=r.n1)
        assert r7.n1 == r.n1 and np.array_equal(r7.x, r.x)
        n1s.append(r.n1)
    assert n1s == sorted(n1s)
    # the FP64 phase does not depend on dot_acc: eps1 > 1 gives FP64-only bits
    r2 = oracle.solve(a, b, 2.0, 1e-10, dot_acc=1)
    rd = oracle.solve(a, b, oracle.EPS1_NONE, 1e-10)
    assert r2.n1 == 0 and np.array_equal(r2.x, rd.x)


def test_dot_acc_out_of_range_is_einval():
    a = W.poisson2d(8)
    _, b = W.rhs(a, seed=0)
    assert oracle.solve(a, b, 1e-4, 1e-10, dot_acc=2).status == oracle.EINVAL


# --------------------------------------------------- CG-Lanczos kappa-hat --

def test_lanczos_kappa_poisson_closed_form():
    """2D 5-point Poisson on 64^2: lambda = 8 sin^2(pi/130) ... 8 cos^2(pi/130),
    kappa = cot^2(pi/130)."""
    a = W.poisson2d(64)
    _, b = W.rhs(a, seed=0)
    kap, lmin, lmax, k = oracle.lanczos_kappa(a, b, 1e-10)
    assert k > 100
    assert abs(lmin / (8 * math.sin(math.pi / 130) ** 2) - 1) < 1e-4
    assert abs(lmax / (8 * math.cos(math.pi / 130) ** 2) - 1) < 1e-4
    assert abs(kap / (1 / math.tan(math.pi / 130) ** 2) - 1) < 2e-4


def test_lanczos_kappa_diagonal_spectrum_is_exact():
    """A diagonal matrix with n distinct eigenvalues and b with no zero
    component: n CG steps span the whole space, so T_n has exactly A's
    eigenvalues."""
    eig = np.linspace(1.0, 40.0, 12)
    a = W.CSR.from_scipy(np.diag(eig))
    b = np.ones(12)
    kap, lmin, lmax, k = oracle.lanczos_kappa(a, b, 1e-14)
    assert abs(lmin - 1.0) < 1e-8 and abs(lmax - 40.0) < 1e-8 and abs(kap - 40.0) < 1e-7


# ------------------------------------------------------- threaded row loops --

@pytest.mark.parametrize("eps1", [oracle.EPS1_NONE, 1e-5])
def test_threaded_row_loops_give_the_same_bits(eps1):
    a = W.varcoef3d(20, seed=1)
    _, b = W.rhs(a, seed=1)
    oracle.set_threads(1)
    r1 = oracle.solve(a, b, eps1, 1e-10)
    oracle.set_threads(4)
    try:
        r4 = oracle.solve(a, b, eps1, 1e-10)
    finally:
        oracle.set_threads(1)
    assert (r1.n1, r1.n2, r1.relres_final_true) == (r4.n1, r4.n2, r4.relres_final_true)
    assert np.array_equal(r1.x, r4.x)


def test_lanczos_iterate_is_the_fp64_only_cg_iterate():
    """The CG run behind kappa-hat is FP64-only CG from 0: its iterate is the
    oracle solve's, bit for bit, when the final check passes at once."""
    a = W.varcoef3d(16, seed=2)
    _, b = W.rhs(a, seed=2)
    kap, lmin, lmax, k, x = oracle.lanczos_kappa(a, b, 1e-10, want_x=True)
    r = oracle.solve(a, b, oracle.EPS1_NONE, 1e-10)
    assert r.status == oracle.OK and r.restarts == 0 and r.n2 == k
    assert np.array_equal(r.x, x)
    assert lmin > 0 and kap == lmax / lmin
