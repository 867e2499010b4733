"""MI355X (gfx950) restarted mixed-precision CG (arXiv 2412.08059).

The work runs in ``libmpcg.so`` (hand-written HIP kernels behind the C ABI in
include/mpcg.h).  This package adds a ctypes binding (``capi``) and a small
torch-facing wrapper: torch supplies device memory and the stream, nothing
else.
"""

from __future__ import annotations

import os

from . import capi  # noqa: F401  (raises ImportError when the library is not built)
from .capi import (  # noqa: F401
    MPCG_EPS1_AUTO,
    MPCG_EPS1_NONE,
    MPCG_OK,
    MpcgError,
    mpcg_csr,
    mpcg_options,
)

DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "knn_model.txt")
# the autotuner's frozen table (paper_2412_08059_amd/autotune.py writes it)
DEFAULT_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.txt")


def _load_tuning(ctx, tuning):
    path = DEFAULT_TUNING if tuning == "default" else tuning
    if path and os.path.exists(path):
        st = capi.mpcg_load_tuning(ctx, path)
        if st != MPCG_OK:
            raise MpcgError(st, f"mpcg_load_tuning({path})")


class DeviceCSR:
    """CSR matrix resident on the GPU (torch tensors) plus its C descriptor."""

    def __init__(self, row_ptr, col, val, n: int, row_ptr_i64: bool = False):
        self.row_ptr, self.col, self.val, self.n = row_ptr, col, val, int(n)
        self.nnz = int(col.numel())
        self.desc = mpcg_csr(self.n, self.nnz, row_ptr.data_ptr(), 1 if row_ptr_i64 else 0, 0,
                             col.data_ptr() if self.nnz else 0, val.data_ptr() if self.nnz else 0)

    @staticmethod
    def from_host(a, device="cuda", row_ptr_i64: bool = False) -> "DeviceCSR":
        import numpy as np
        import torch
        rp_dtype = np.int64 if row_ptr_i64 else np.int32
        rp = torch.from_numpy(np.ascontiguousarray(a.row_ptr, dtype=rp_dtype)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(a.col, dtype=np.int32)).to(device)
        val = torch.from_numpy(np.ascontiguousarray(a.val, dtype=np.float64)).to(device)
        return DeviceCSR(rp, col, val, a.n, row_ptr_i64)


class Solver:
    """One library context bound to the current torch stream, with its own
    workspace tensor sized for systems up to (n_max, nnz_max)."""

    def __init__(self, n_max: int, nnz_max: int, *, k0: int = 20, knn_k: int = 0, tol_mode: int = 0,
                 max_restarts: int = 5, graph_iters: int = 0, maxit1: int = 0, maxit2: int = 0,
                 model: str | None = None, precond: int = 0, dot_acc: int = 0, spmv_variant: int = 0,
                 bfs_mode: int = 0, tuning: str | dict | None = "default", device="cuda"):
        """precond = 1: Jacobi-preconditioned stages (M = diag(A)); dot_acc = 1:
        FP32-accumulated FP32-phase dot products; spmv_variant / bfs_mode: see
        mpcg_options in include/mpcg.h.  tuning: "default" (the packaged
        table, if present), a table path, a dict of mpcg_tuning fields used
        for every matrix, or None (built-in defaults)."""
        import torch
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        opt = mpcg_options(k0, knn_k, tol_mode, max_restarts, graph_iters, precond, maxit1, maxit2, dot_acc,
                           spmv_variant, bfs_mode, 0)
        self.ctx = capi.mpcg_create(opt, self.stream.cuda_stream)
        self.set_tuning(tuning)
        nbytes = capi.mpcg_workspace_size(self.ctx, max(1, n_max), max(0, nnz_max))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        st = capi.mpcg_set_workspace(self.ctx, self.workspace.data_ptr(), nbytes)
        if st != MPCG_OK:
            raise MpcgError(st, "mpcg_set_workspace")
        if model:
            st = capi.mpcg_load_model(self.ctx, model)
            if st != MPCG_OK:
                raise MpcgError(st, f"mpcg_load_model({model})")

    def set_tuning(self, tuning):
        """A table path ("default": the packaged one), a dict of mpcg_tuning
        fields for every matrix, or None (clears explicit values)."""
        if isinstance(tuning, dict):
            st = capi.mpcg_set_tuning(self.ctx, tuning)
            if st != MPCG_OK:
                raise MpcgError(st, "mpcg_set_tuning")
        else:
            capi.mpcg_set_tuning(self.ctx, None)
            _load_tuning(self.ctx, tuning)

    def tuning_for(self, n: int, nnz: int, band: int) -> dict:
        st, t = capi.mpcg_get_tuning(self.ctx, n, nnz, band)
        if st != MPCG_OK:
            raise MpcgError(st, "mpcg_get_tuning")
        return t.as_dict()

    def close(self):
        if getattr(self, "ctx", None):
            capi.mpcg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, A: DeviceCSR, b, eps1: float, eps2: float = 1e-10, x=None):
        """Returns (status, x, stats); x is a float64 device tensor."""
        import torch
        if x is None:
            x = torch.empty(A.n, dtype=torch.float64, device=self.device)
        st, stats = capi.mpcg_solve(self.ctx, A.desc, b.data_ptr(), x.data_ptr(), eps1, eps2)
        return st, x, stats

    def solve_jacobi(self, A: DeviceCSR, b, eps1: float, eps2: float = 1e-10, x=None):
        """Algorithm I with the Jacobi method (mpcg_solve_jacobi); returns (status, x, stats)."""
        import torch
        if x is None:
            x = torch.empty(A.n, dtype=torch.float64, device=self.device)
        st, stats = capi.mpcg_solve_jacobi(self.ctx, A.desc, b.data_ptr(), x.data_ptr(), eps1, eps2)
        return st, x, stats

    def features(self, A: DeviceCSR, b, k0: int = 20):
        return capi.mpcg_features(self.ctx, A.desc, b.data_ptr(), k0)

    def spmv(self, A: DeviceCSR, x, precision: int = 64):
        import torch
        dt = torch.float64 if precision == 64 else torch.float32
        y = torch.empty(A.n, dtype=dt, device=self.device)
        st = capi.mpcg_spmv(self.ctx, A.desc, precision, x.data_ptr(), y.data_ptr())
        return st, y

    def bfs(self, A: DeviceCSR, src: int):
        import torch
        dist = torch.empty(A.n, dtype=torch.int32, device=self.device)
        st, ecc, far = capi.mpcg_bfs(self.ctx, A.desc, src, dist.data_ptr())
        return st, dist, ecc, far

    def diameter_multi(self, A: DeviceCSR, starts, q: float = 0.9):
        """Multi-start 2BFS and the effective-diameter estimate (mpcg_diameter_multi)."""
        return capi.mpcg_diameter_multi(self.ctx, A.desc, list(starts), q)


class BatchSolver:
    """Batched / continuously admitted solves (the mpcg_batch_* entry points).

    Owns a library context whose engine thread runs on a stream of its own,
    and the batch arena (one uint8 tensor).  Submitted systems keep their
    tensors referenced here until their result has been polled."""

    def __init__(self, max_rows: int, max_entries: int, max_systems: int, *, k0: int = 20, knn_k: int = 0,
                 tol_mode: int = 0, max_restarts: int = 5, maxit1: int = 0, maxit2: int = 0,
                 model: str | None = DEFAULT_MODEL, dot_acc: int = 0, tuning: str | dict | None = "default",
                 device="cuda"):
        """tuning: as for Solver; its batch_* fields set the engine's schedule."""
        import torch
        self.device = torch.device(device)
        opt = mpcg_options(k0, knn_k, tol_mode, max_restarts, 0, 0, maxit1, maxit2, dot_acc)
        self.ctx = capi.mpcg_create(opt, torch.cuda.current_stream(self.device).cuda_stream)
        if isinstance(tuning, dict):
            st = capi.mpcg_set_tuning(self.ctx, tuning)
            if st != MPCG_OK:
                raise MpcgError(st, "mpcg_set_tuning")
        else:
            _load_tuning(self.ctx, tuning)
        if model:
            st = capi.mpcg_load_model(self.ctx, model)
            if st != MPCG_OK:
                raise MpcgError(st, f"mpcg_load_model({model})")
        nbytes = capi.mpcg_batch_workspace_size(self.ctx, max_rows, max_entries, max_systems)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        st = capi.mpcg_batch_set_workspace(self.ctx, self.arena.data_ptr(), nbytes, max_rows, max_entries,
                                           max_systems)
        if st != MPCG_OK:
            raise MpcgError(st, "mpcg_batch_set_workspace")
        self.live = {}

    def submit(self, systems):
        """systems: iterable of (DeviceCSR, b, x, eps1, eps2); returns the ids."""
        import torch
        systems = list(systems)
        torch.cuda.current_stream(self.device).synchronize()   # inputs complete before the engine reads them
        reqs = [capi.mpcg_request(A.desc, b.data_ptr(), x.data_ptr(), float(e1), float(e2), None)
                for (A, b, x, e1, e2) in systems]
        st, ids = capi.mpcg_batch_submit(self.ctx, reqs)
        if st != MPCG_OK:
            raise MpcgError(st, "mpcg_batch_submit")
        for rid, sysd in zip(ids, systems):
            self.live[rid] = sysd
        return ids

    def poll(self, cap: int = 256):
        """Finished requests as (id, stats, x); non-blocking."""
        st, done = capi.mpcg_batch_poll(self.ctx, cap)
        if st != MPCG_OK:
            raise MpcgError(st, "mpcg_batch_poll")
        out = []
        for rid, stats in done:
            sysd = self.live.pop(rid, None)
            out.append((rid, stats, sysd[2] if sysd else None))
        return out

    def wait_all(self, ids, timeout_s: float = 600.0, sleep_s: float = 0.0005):
        """Polls until every id in `ids` is reported; returns {id: (stats, x)}."""
        import time
        want, got = set(ids), {}
        t0 = time.perf_counter()
        while want:
            for rid, stats, x in self.poll():
                if rid in want:
                    want.discard(rid)
                    got[rid] = (stats, x)
            if want:
                if time.perf_counter() - t0 > timeout_s:
                    raise TimeoutError(f"{len(want)} batch requests not finished after {timeout_s} s")
                time.sleep(sleep_s)
        return got

    def cancel(self, rid: int) -> int:
        return capi.mpcg_batch_cancel(self.ctx, rid)

    def load(self):
        st, q, a = capi.mpcg_batch_load(self.ctx)
        return q, a

    def close(self):
        if getattr(self, "ctx", None):
            capi.mpcg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
