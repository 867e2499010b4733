"""mpcg_solve_noalloc (the solve on the library's built-in device array,
through the C ABI) against mpcg_solve on the context's arena: the same
kernels on the same inputs, so counts, flags and x must be the same bits.
Two calls in a row, the second on a smaller system, so that the array still
holds the first call's contents when the second starts; then a system larger
than the array is refused with ENOMEM."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

NOALLOC_BYTES = 160 << 20


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _same(torch_mod, solver, a, b, eps1):
    from paper_2412_08059_amd import DeviceCSR, capi
    A = DeviceCSR.from_host(a)
    B = torch_mod.from_numpy(b).cuda()
    st0, x0, s0 = solver.solve(A, B, eps1, 1e-10)
    x1 = torch_mod.full((a.n,), float("nan"), dtype=torch_mod.float64, device="cuda")
    st1, s1 = capi.mpcg_solve_noalloc(solver.ctx, A.desc, B.data_ptr(), x1.data_ptr(), eps1, 1e-10)
    print(f"noalloc n={a.n} eps1={eps1}: arena n1={s0.n1} n2={s0.n2}, noalloc n1={s1.n1} n2={s1.n2}", flush=True)
    assert st0 == 0 and st1 == 0
    assert (s0.n1, s0.n2, s0.restarts, s0.flags, s0.eps1_class) == (s1.n1, s1.n2, s1.restarts, s1.flags,
                                                                       s1.eps1_class)
    assert s0.relres_final_true == s1.relres_final_true <= 1e-10
    assert np.array_equal(x0.cpu().numpy().view(np.uint64), x1.cpu().numpy().view(np.uint64))


def test_noalloc_solve_equals_arena_solve(torch_mod):
    from paper_2412_08059_amd import DEFAULT_MODEL, DeviceCSR, Solver, capi
    big = W.varcoef3d(56, seed=1)          # 175,616 rows
    small = W.poisson2d(64)
    solver = Solver(big.n, big.nnz, model=DEFAULT_MODEL)
    try:
        assert capi.mpcg_workspace_size(solver.ctx, big.n, big.nnz) <= NOALLOC_BYTES
        _, bb = W.rhs(big, seed=2)
        _, bs = W.rhs(small, seed=3)
        _same(torch_mod, solver, big, bb, 1e-5)
        _same(torch_mod, solver, small, bs, 0.0)     # second call, smaller, Algorithm II
        _same(torch_mod, solver, small, bs, -1.0)
        # a system whose workspace exceeds the array: refused before any access
        n_big = 2_000_000
        assert capi.mpcg_workspace_size(solver.ctx, n_big, 7 * n_big) > NOALLOC_BYTES
        A = DeviceCSR.from_host(small)
        desc = capi.mpcg_csr(n_big, 7 * n_big, A.desc.row_ptr, 0, 0, A.desc.col_idx, A.desc.val)
        x = torch_mod.empty(small.n, dtype=torch_mod.float64, device="cuda")
        st, _ = capi.mpcg_solve_noalloc(solver.ctx, desc, x.data_ptr(), x.data_ptr(), 1e-4, 1e-10)
        assert st == capi.MPCG_ENOMEM
    finally:
        solver.close()
