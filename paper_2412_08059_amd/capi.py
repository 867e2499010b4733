"""Thin ctypes binding of ``libmpcg.so`` (include/mpcg.h).

Every ``mpcg_*`` function here has the name and argument order of the C entry
point and does argument marshalling only; all of the method runs in the HIP
library.  Device buffers are passed as integer addresses (``tensor.data_ptr()``)
and the stream as ``torch.cuda.current_stream().cuda_stream``.

There is no fallback: if the library is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpcg.so")

MPCG_OK = 0
MPCG_EINVAL = -1
MPCG_ENOTSPD = -2
MPCG_ENOCONV = -3
MPCG_ENOMEM = -4
MPCG_EDEVICE = -5
MPCG_ENONFINITE = -6
MPCG_EBUSY = -7
MPCG_ECANCELED = -8
MPCG_ENOMODEL = -9

MPCG_EPS1_AUTO = 0.0
MPCG_EPS1_NONE = -1.0

MPCG_FLAG_FP32_BREAKDOWN = 1
MPCG_FLAG_FP32_MAXIT = 2
MPCG_FLAG_FINAL_RESTARTED = 4
MPCG_FLAG_KNN_EXACT = 8
MPCG_FLAG_BFS_DIA = 16

EXPORTED = (
    "mpcg_create", "mpcg_destroy", "mpcg_workspace_size", "mpcg_set_workspace", "mpcg_load_model",
    "mpcg_features", "mpcg_select_eps1", "mpcg_solve", "mpcg_solve_noalloc", "mpcg_solve_jacobi", "mpcg_spmv",
    "mpcg_bfs",
    "mpcg_diameter_multi",
    "mpcg_set_tuning", "mpcg_load_tuning", "mpcg_get_tuning",
    "mpcg_last_kernel_ms", "mpcg_time_kernel", "mpcg_strerror",
    "mpcg_batch_workspace_size", "mpcg_batch_set_workspace", "mpcg_batch_submit", "mpcg_batch_poll",
    "mpcg_batch_cancel", "mpcg_batch_load",
)

MPCG_KERNEL_CG_SPMV_F64 = 0
MPCG_KERNEL_CG_SPMV_F32 = 1
MPCG_KERNEL_UPDATE_F64 = 2
MPCG_KERNEL_UPDATE_F32 = 3
MPCG_KERNEL_SPMV_F64 = 4
MPCG_KERNEL_SPMV_F32 = 5
MPCG_KERNEL_JACOBI_F64 = 6
MPCG_KERNEL_JACOBI_F32 = 7


class mpcg_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("row_ptr_is_i64", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class mpcg_features_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("pdiam", ctypes.c_int64),
                ("bfs_t", ctypes.c_int64), ("bfs_u", ctypes.c_int64),
                ("n_components", ctypes.c_int32), ("k0_used", ctypes.c_int32), ("v", ctypes.c_double)]


class mpcg_diam_t(ctypes.Structure):
    _fields_ = [("pdiam", ctypes.c_int64), ("pdiam_multi", ctypes.c_int64), ("eff_diam", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("best_start", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class mpcg_stats(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("eps1_class", ctypes.c_int32), ("status", ctypes.c_int32),
                ("eps1_used", ctypes.c_double), ("relres_sp", ctypes.c_double),
                ("relres_restart_true", ctypes.c_double), ("relres_final_true", ctypes.c_double),
                ("omega_measured", ctypes.c_double), ("I_third", ctypes.c_double),
                ("I_meas", ctypes.c_double), ("t_feat_ms", ctypes.c_double), ("t_sp_ms", ctypes.c_double),
                ("t_dp_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("feat", mpcg_features_t)]


class mpcg_options(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_int32), ("knn_k", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("graph_iters", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("maxit1", ctypes.c_int64), ("maxit2", ctypes.c_int64),
                ("dot_acc", ctypes.c_int32), ("spmv_variant", ctypes.c_int32), ("bfs_mode", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class mpcg_tuning(ctypes.Structure):
    _fields_ = [("sell_batch", ctypes.c_int32), ("sell_whole_batch", ctypes.c_int32),
                ("sell_split", ctypes.c_int32), ("bfs_grid", ctypes.c_int32), ("bfs_grid_shared", ctypes.c_int32),
                ("bfs_persist", ctypes.c_int32), ("batch_group_steps", ctypes.c_int32),
                ("batch_bfs_rounds", ctypes.c_int32), ("batch_small_cap", ctypes.c_int32),
                ("batch_small_levels", ctypes.c_int32), ("batch_level_grid", ctypes.c_int32),
                ("bfs_dia", ctypes.c_int32), ("bfs_dia_tiles", ctypes.c_int32), ("sell_stream", ctypes.c_int32),
                ("batch_runahead", ctypes.c_int32), ("batch_bfs_band", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class mpcg_request(ctypes.Structure):
    _fields_ = [("A", mpcg_csr), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("eps1", ctypes.c_double),
                ("eps2", ctypes.c_double), ("user", ctypes.c_void_p)]


def _load():
    # torch ships its own libamdhip64.so.7; loading torch first makes the
    # library bind to that same HIP runtime instance (one runtime per process,
    # so torch's streams and allocations are valid handles here).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2412_08059_amd.build.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mpcg_create": ([ctypes.POINTER(P), ctypes.POINTER(mpcg_options), P], I32),
        "mpcg_destroy": ([P], I32),
        "mpcg_workspace_size": ([P, I64, I64, ctypes.POINTER(ctypes.c_size_t)], I32),
        "mpcg_set_workspace": ([P, P, ctypes.c_size_t], I32),
        "mpcg_load_model": ([P, ctypes.c_char_p], I32),
        "mpcg_features": ([P, ctypes.POINTER(mpcg_csr), P, I32, ctypes.POINTER(mpcg_features_t)], I32),
        "mpcg_select_eps1": ([P, ctypes.POINTER(mpcg_features_t), ctypes.POINTER(D),
                              ctypes.POINTER(I32)], I32),
        "mpcg_solve": ([P, ctypes.POINTER(mpcg_csr), P, P, D, D, ctypes.POINTER(mpcg_stats)], I32),
        "mpcg_solve_noalloc": ([P, ctypes.POINTER(mpcg_csr), P, P, D, D, ctypes.POINTER(mpcg_stats)], I32),
        "mpcg_solve_jacobi": ([P, ctypes.POINTER(mpcg_csr), P, P, D, D, ctypes.POINTER(mpcg_stats)], I32),
        "mpcg_spmv": ([P, ctypes.POINTER(mpcg_csr), I32, P, P], I32),
        "mpcg_bfs": ([P, ctypes.POINTER(mpcg_csr), I64, P, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "mpcg_diameter_multi": ([P, ctypes.POINTER(mpcg_csr), ctypes.POINTER(I32), I32, D,
                                 ctypes.POINTER(mpcg_diam_t)], I32),
        "mpcg_set_tuning": ([P, ctypes.POINTER(mpcg_tuning)], I32),
        "mpcg_load_tuning": ([P, ctypes.c_char_p], I32),
        "mpcg_get_tuning": ([P, I64, I64, I64, ctypes.POINTER(mpcg_tuning)], I32),
        "mpcg_last_kernel_ms": ([P, ctypes.POINTER(D)], I32),
        "mpcg_time_kernel": ([P, ctypes.POINTER(mpcg_csr), I32, I32, ctypes.POINTER(D)], I32),
        "mpcg_strerror": ([I32], ctypes.c_char_p),
        "mpcg_batch_workspace_size": ([P, I64, I64, I32, ctypes.POINTER(ctypes.c_size_t)], I32),
        "mpcg_batch_set_workspace": ([P, P, ctypes.c_size_t, I64, I64, I32], I32),
        "mpcg_batch_submit": ([P, ctypes.POINTER(mpcg_request), I32, ctypes.POINTER(ctypes.c_uint64)], I32),
        "mpcg_batch_poll": ([P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(mpcg_stats), I32,
                             ctypes.POINTER(I32)], I32),
        "mpcg_batch_cancel": ([P, ctypes.c_uint64], I32),
        "mpcg_batch_load": ([P, ctypes.POINTER(I32), ctypes.POINTER(I32)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


class MpcgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {mpcg_strerror(status)} ({status})")


def _check(st: int, where: str):
    if st != MPCG_OK:
        raise MpcgError(st, where)


# ----------------------------------------------------------- raw wrappers --

def mpcg_strerror(status: int) -> str:
    return lib.mpcg_strerror(int(status)).decode()


def mpcg_create(opt: mpcg_options | None = None, stream: int | None = None) -> int:
    ctx = ctypes.c_void_p()
    st = lib.mpcg_create(ctypes.byref(ctx), ctypes.byref(opt) if opt is not None else None,
                         ctypes.c_void_p(stream) if stream else None)
    _check(st, "mpcg_create")
    return ctx.value


def mpcg_destroy(ctx: int) -> int:
    return lib.mpcg_destroy(ctypes.c_void_p(ctx))


def mpcg_workspace_size(ctx: int, n: int, nnz: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib.mpcg_workspace_size(ctypes.c_void_p(ctx), n, nnz, ctypes.byref(b)), "mpcg_workspace_size")
    return b.value


def mpcg_set_workspace(ctx: int, ptr: int, nbytes: int) -> int:
    return lib.mpcg_set_workspace(ctypes.c_void_p(ctx), ctypes.c_void_p(ptr), nbytes)


def mpcg_load_model(ctx: int, path: str) -> int:
    return lib.mpcg_load_model(ctypes.c_void_p(ctx), path.encode())


def mpcg_features(ctx: int, A: mpcg_csr, b_ptr: int, k0: int):
    f = mpcg_features_t()
    st = lib.mpcg_features(ctypes.c_void_p(ctx), ctypes.byref(A), ctypes.c_void_p(b_ptr), k0,
                           ctypes.byref(f))
    return st, f


def mpcg_select_eps1(ctx: int, f: mpcg_features_t):
    e = ctypes.c_double(0.0)
    t = ctypes.c_int32(0)
    st = lib.mpcg_select_eps1(ctypes.c_void_p(ctx), ctypes.byref(f), ctypes.byref(e), ctypes.byref(t))
    return st, e.value, t.value


def mpcg_solve(ctx: int, A: mpcg_csr, b_ptr: int, x_ptr: int, eps1: float, eps2: float):
    s = mpcg_stats()
    st = lib.mpcg_solve(ctypes.c_void_p(ctx), ctypes.byref(A), ctypes.c_void_p(b_ptr),
                        ctypes.c_void_p(x_ptr), float(eps1), float(eps2), ctypes.byref(s))
    return st, s


def mpcg_solve_noalloc(ctx: int, A: mpcg_csr, b_ptr: int, x_ptr: int, eps1: float, eps2: float):
    s = mpcg_stats()
    st = lib.mpcg_solve_noalloc(ctypes.c_void_p(ctx), ctypes.byref(A), ctypes.c_void_p(b_ptr),
                                ctypes.c_void_p(x_ptr), float(eps1), float(eps2), ctypes.byref(s))
    return st, s


def mpcg_set_tuning(ctx: int, t) -> int:
    """t: an mpcg_tuning, a dict of its fields (the rest from the defaults
    mpcg_get_tuning reports for an empty context), or None to clear."""
    if t is None:
        return lib.mpcg_set_tuning(ctypes.c_void_p(ctx), None)
    if isinstance(t, dict):
        st, base = mpcg_get_tuning(ctx, 1, 1, 0)
        for k, v in t.items():
            setattr(base, k, int(v))
        t = base
    return lib.mpcg_set_tuning(ctypes.c_void_p(ctx), ctypes.byref(t))


def mpcg_load_tuning(ctx: int, path: str) -> int:
    return lib.mpcg_load_tuning(ctypes.c_void_p(ctx), path.encode())


def mpcg_get_tuning(ctx: int, n: int, nnz: int, band: int):
    t = mpcg_tuning()
    st = lib.mpcg_get_tuning(ctypes.c_void_p(ctx), int(n), int(nnz), int(band), ctypes.byref(t))
    return st, t


def mpcg_spmv(ctx: int, A: mpcg_csr, precision: int, x_ptr: int, y_ptr: int) -> int:
    return lib.mpcg_spmv(ctypes.c_void_p(ctx), ctypes.byref(A), precision, ctypes.c_void_p(x_ptr),
                         ctypes.c_void_p(y_ptr))


def mpcg_solve_jacobi(ctx: int, A: mpcg_csr, b_ptr: int, x_ptr: int, eps1: float, eps2: float):
    s = mpcg_stats()
    st = lib.mpcg_solve_jacobi(ctypes.c_void_p(ctx), ctypes.byref(A), ctypes.c_void_p(b_ptr),
                               ctypes.c_void_p(x_ptr), float(eps1), float(eps2), ctypes.byref(s))
    return st, s


def mpcg_bfs(ctx: int, A: mpcg_csr, src: int, dist_ptr: int):
    ecc = ctypes.c_int64(0)
    far = ctypes.c_int64(0)
    st = lib.mpcg_bfs(ctypes.c_void_p(ctx), ctypes.byref(A), src, ctypes.c_void_p(dist_ptr),
                      ctypes.byref(ecc), ctypes.byref(far))
    return st, ecc.value, far.value


def mpcg_diameter_multi(ctx: int, A: mpcg_csr, starts, q: float = 0.9):
    arr = (ctypes.c_int32 * max(1, len(starts)))(*[int(v) for v in starts])
    out = mpcg_diam_t()
    st = lib.mpcg_diameter_multi(ctypes.c_void_p(ctx), ctypes.byref(A), arr, len(starts), float(q),
                                 ctypes.byref(out))
    return st, out


def mpcg_last_kernel_ms(ctx: int) -> float:
    ms = ctypes.c_double(0.0)
    _check(lib.mpcg_last_kernel_ms(ctypes.c_void_p(ctx), ctypes.byref(ms)), "mpcg_last_kernel_ms")
    return ms.value


def mpcg_time_kernel(ctx: int, A: mpcg_csr, kernel: int, reps: int) -> float:
    ms = ctypes.c_double(0.0)
    _check(lib.mpcg_time_kernel(ctypes.c_void_p(ctx), ctypes.byref(A), kernel, reps, ctypes.byref(ms)),
           "mpcg_time_kernel")
    return ms.value


def mpcg_batch_workspace_size(ctx: int, max_rows: int, max_entries: int, max_systems: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib.mpcg_batch_workspace_size(ctypes.c_void_p(ctx), max_rows, max_entries, max_systems,
                                         ctypes.byref(b)), "mpcg_batch_workspace_size")
    return b.value


def mpcg_batch_set_workspace(ctx: int, ptr: int, nbytes: int, max_rows: int, max_entries: int,
                             max_systems: int) -> int:
    return lib.mpcg_batch_set_workspace(ctypes.c_void_p(ctx), ctypes.c_void_p(ptr), nbytes, max_rows,
                                        max_entries, max_systems)


def mpcg_batch_submit(ctx: int, reqs) -> tuple[int, list[int]]:
    n = len(reqs)
    arr = (mpcg_request * max(n, 1))(*reqs)
    ids = (ctypes.c_uint64 * max(n, 1))()
    st = lib.mpcg_batch_submit(ctypes.c_void_p(ctx), arr, n, ids)
    return st, [int(ids[i]) for i in range(n)] if st == MPCG_OK else []


def mpcg_batch_poll(ctx: int, cap: int = 256):
    ids = (ctypes.c_uint64 * cap)()
    stats = (mpcg_stats * cap)()
    nd = ctypes.c_int32(0)
    st = lib.mpcg_batch_poll(ctypes.c_void_p(ctx), ids, stats, cap, ctypes.byref(nd))
    return st, [(int(ids[i]), stats[i]) for i in range(nd.value)]


def mpcg_batch_cancel(ctx: int, rid: int) -> int:
    return lib.mpcg_batch_cancel(ctypes.c_void_p(ctx), rid)


def mpcg_batch_load(ctx: int):
    q = ctypes.c_int32(0)
    a = ctypes.c_int32(0)
    st = lib.mpcg_batch_load(ctypes.c_void_p(ctx), ctypes.byref(q), ctypes.byref(a))
    return st, q.value, a.value
