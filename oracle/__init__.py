"""CPU oracle for the restarted mixed-precision CG method (arXiv 2412.08059).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the bench may import this package; the product library never does.  The
arithmetic lives in ``mpcg_oracle.c`` (plain C, FP64 unless the method fixes
FP32, no FMA contraction); this module only marshals numpy arrays.

Functions and the passages they follow:
  spmv64 / spmv32     the product A d of the CG iteration (eq. 16 cost model:
                      one multiply-add per stored entry, an fma chain per row).
  bfs                 breadth-first search over the matrix graph (2BFS section).
  pseudo_diameter     2BFS per connected component, maximum over components.
  knn_select          weighted kNN with min-max normalisation, squared
                      Euclidean search and 1/rho weights (eq. 22-23).
  solve               Algorithm I (explicit eps1), Algorithm II (eps1 = AUTO)
                      and FP64-only CG (eps1 = NONE).
  cg64_directions     search directions of FP64 CG (A-orthogonality pin).
  cg_true_residuals   true residual history of plain SP or DP CG (Fig. 2).
  lanczos_kappa       condition-number estimate from the CG-Lanczos
                      tridiagonal of an FP64 CG run (gates the x-parity bar).
  set_threads         host threads for the row loops (products and
                      element-wise updates; same bits as one thread).
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

from .knn_model import KnnModel, load_model, save_model  # noqa: F401
from . import cost  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EPS1_AUTO = 0.0
EPS1_NONE = -1.0

OK, EINVAL, ENOTSPD, ENOCONV, ENOMEM, ENONFINITE, ENOMODEL = 0, -1, -2, -3, -4, -6, -9
FLAG_FP32_BREAKDOWN, FLAG_FP32_MAXIT, FLAG_FINAL_RESTARTED, FLAG_KNN_EXACT = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                               "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("knn_k", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("dot_acc", ctypes.c_int32),
                ("maxit1", ctypes.c_int64), ("maxit2", ctypes.c_int64)]


class _Model(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int64), ("feat", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("fmin", ctypes.c_void_p), ("fmax", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("mask", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("flags", ctypes.c_int32), ("k0_used", ctypes.c_int32),
                ("eps1_class", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("eps1_used", ctypes.c_double), ("v", ctypes.c_double), ("beta_b", ctypes.c_double),
                ("relres_sp", ctypes.c_double), ("relres_restart_true", ctypes.c_double),
                ("relres_final_true", ctypes.c_double),
                ("ell", ctypes.c_int64), ("bfs_t", ctypes.c_int64), ("bfs_u", ctypes.c_int64),
                ("ncomp", ctypes.c_int64)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.or_spmv64.argtypes = [I64, P, P, P, P, P]
        lib.or_spmv32.argtypes = [I64, P, P, P, P, P]
        lib.or_bfs.argtypes = [I64, P, P, I64, P]
        lib.or_bfs.restype = ctypes.c_int32
        lib.or_pseudo_diameter.argtypes = [I64, P, P, P]
        lib.or_pseudo_diameter.restype = ctypes.c_int
        lib.or_jacobi_solve.argtypes = [I64, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(_Opts), ctypes.POINTER(_Stats)]
        lib.or_jacobi_solve.restype = ctypes.c_int
        lib.or_diameter_multi.argtypes = [I64, P, P, P, ctypes.c_int32, ctypes.c_double, P]
        lib.or_diameter_multi.restype = ctypes.c_int
        lib.or_knn_select.argtypes = [ctypes.POINTER(_Model), P, ctypes.c_int32, P, P]
        lib.or_knn_select.restype = ctypes.c_int
        lib.or_solve.argtypes = [I64, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(_Opts), ctypes.POINTER(_Model), ctypes.POINTER(_Stats)]
        lib.or_solve.restype = ctypes.c_int
        lib.or_cg64_directions.argtypes = [I64, P, P, P, P, I64, P]
        lib.or_cg64_directions.restype = I64
        lib.or_cg_true_residuals.argtypes = [ctypes.c_int32, I64, P, P, P, P, I64, P]
        lib.or_cg_lanczos.argtypes = [I64, P, P, P, P, ctypes.c_double, I64, P, P, P]
        lib.or_cg_lanczos.restype = I64
        lib.or_set_threads.argtypes = [ctypes.c_int32]
        lib.or_get_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(a):
    rp = np.ascontiguousarray(a.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(a.col, dtype=np.int32)
    val = np.ascontiguousarray(a.val, dtype=np.float64)
    return rp, col, val


def spmv64(a, x) -> np.ndarray:
    rp, col, val = _csr_arrays(a)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(a.n, dtype=np.float64)
    _L().or_spmv64(a.n, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def spmv32(a, x) -> np.ndarray:
    """FP32 product with A~ = float32(A) (round to nearest even)."""
    rp, col, val = _csr_arrays(a)
    v32 = val.astype(np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(a.n, dtype=np.float32)
    _L().or_spmv32(a.n, _p(rp), _p(col), _p(v32), _p(x), _p(y))
    return y


def bfs(a, src: int):
    """Distances from src (int32, -1 when unreached) and the eccentricity."""
    rp, col, _ = _csr_arrays(a)
    dist = np.empty(a.n, dtype=np.int32)
    ecc = _L().or_bfs(a.n, _p(rp), _p(col), int(src), _p(dist))
    return dist, int(ecc)


def pseudo_diameter(a):
    """(ell, t, u, n_components) of the 2BFS procedure, maximised over components."""
    rp, col, _ = _csr_arrays(a)
    out = np.zeros(4, dtype=np.int64)
    st = _L().or_pseudo_diameter(a.n, _p(rp), _p(col), _p(out))
    if st != OK:
        raise ValueError(f"or_pseudo_diameter status {st}")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3])


def solve_jacobi(a, b, eps1: float, eps2: float = 1e-10, *, tol_mode: int = 0, maxit1: int = 0,
                 maxit2: int = 0) -> OracleResult:
    """Algorithm I with the Jacobi method: FP32 stage to eps1 (eps1 = -1:
    none), then FP64 from float64(x~) to eps2."""
    rp, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(a.n, dtype=np.float64)
    opts = _Opts(20, tol_mode, 0, 0, 0, 0, maxit1, maxit2)
    st = _Stats()
    status = _L().or_jacobi_solve(a.n, _p(rp), _p(col), _p(val), _p(b), _p(x), float(eps1), float(eps2),
                                  ctypes.byref(opts), ctypes.byref(st))
    return OracleResult(status=status, x=x, n1=st.n1, n2=st.n2, restarts=0, flags=st.flags, k0_used=0,
                        eps1_class=-1, eps1_used=st.eps1_used, v=0.0, beta_b=0.0, relres_sp=st.relres_sp,
                        relres_restart_true=0.0, relres_final_true=st.relres_final_true, ell=0, bfs_t=0,
                        bfs_u=0, ncomp=0)


def diameter_multi(a, starts, q: float = 0.9):
    """(pdiam, pdiam_multi, eff_diam, pairs, best_start): 2BFS repeated from
    `starts` and the effective diameter over the starts' distances."""
    rp, col, _ = _csr_arrays(a)
    s = np.ascontiguousarray(np.asarray(starts, dtype=np.int32))
    if s.size == 0:
        s = np.zeros(1, dtype=np.int32)
        cnt = 0
    else:
        cnt = int(s.size)
    out = np.zeros(5, dtype=np.int64)
    st = _L().or_diameter_multi(a.n, _p(rp), _p(col), _p(s), cnt, float(q), _p(out))
    if st != OK:
        raise ValueError(f"or_diameter_multi status {st}")
    return tuple(int(v) for v in out)


def _model_struct(m: KnnModel):
    feat = np.ascontiguousarray(m.feat, dtype=np.float64)
    lab = np.ascontiguousarray(m.label, dtype=np.int32)
    fmin = np.ascontiguousarray(m.fmin, dtype=np.float64)
    fmax = np.ascontiguousarray(m.fmax, dtype=np.float64)
    s = _Model(feat.shape[0], _p(feat).value, _p(lab).value, _p(fmin).value, _p(fmax).value,
               int(m.k), int(m.mask))
    return s, (feat, lab, fmin, fmax)


def knn_select(m: KnnModel, chi, k: int = 0):
    """Class t (2..7), the six class scores and the zero-distance flag."""
    s, keep = _model_struct(m)
    q = np.ascontiguousarray(chi, dtype=np.float64)
    scores = np.zeros(6, dtype=np.float64)
    ex = ctypes.c_int32(0)
    t = _L().or_knn_select(ctypes.byref(s), _p(q), int(k), _p(scores), ctypes.byref(ex))
    del keep
    if t < 0:
        raise ValueError(f"or_knn_select status {t}")
    return int(t), scores, bool(ex.value)


@dataclasses.dataclass
class OracleResult:
    status: int
    x: np.ndarray
    n1: int
    n2: int
    restarts: int
    flags: int
    k0_used: int
    eps1_class: int
    eps1_used: float
    v: float
    beta_b: float
    relres_sp: float
    relres_restart_true: float
    relres_final_true: float
    ell: int
    bfs_t: int
    bfs_u: int
    ncomp: int


def solve(a, b, eps1: float, eps2: float = 1e-10, *, k0: int = 20, tol_mode: int = 0,
          max_restarts: int = 5, maxit1: int = 0, maxit2: int = 0, knn_k: int = 0,
          model: KnnModel | None = None, precond: int = 0, dot_acc: int = 0,
          x0=None) -> OracleResult:
    """precond = 1: every CG stage preconditioned with M = diag(A) (Jacobi).
    dot_acc = 1: FP32-phase dot products accumulate in FP32 (else FP64).
    x0: initial guess of the first stage (float32(x0) for the FP32 stage,
    x0 for FP64-only CG); None is zero."""
    rp, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(a.n, dtype=np.float64)
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    opts = _Opts(k0, tol_mode, max_restarts, knn_k, precond, dot_acc, maxit1, maxit2)
    st = _Stats()
    keep = None
    mp = None
    if model is not None:
        ms, keep = _model_struct(model)
        mp = ctypes.byref(ms)
    status = _L().or_solve(a.n, _p(rp), _p(col), _p(val), _p(b), None if x0a is None else _p(x0a), _p(x),
                           float(eps1), float(eps2), ctypes.byref(opts), mp, ctypes.byref(st))
    del keep
    return OracleResult(status=status, x=x, n1=st.n1, n2=st.n2, restarts=st.restarts, flags=st.flags,
                        k0_used=st.k0_used, eps1_class=st.eps1_class, eps1_used=st.eps1_used, v=st.v,
                        beta_b=st.beta_b, relres_sp=st.relres_sp,
                        relres_restart_true=st.relres_restart_true,
                        relres_final_true=st.relres_final_true, ell=st.ell, bfs_t=st.bfs_t,
                        bfs_u=st.bfs_u, ncomp=st.ncomp)


def cg64_directions(a, b, nd: int) -> np.ndarray:
    rp, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros((nd, a.n), dtype=np.float64)
    got = _L().or_cg64_directions(a.n, _p(rp), _p(col), _p(val), _p(b), nd, _p(out))
    return out[:got]


def cg_true_residuals(a, b, prec: int, iters: int) -> np.ndarray:
    rp, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros(iters + 1, dtype=np.float64)
    _L().or_cg_true_residuals(int(prec), a.n, _p(rp), _p(col), _p(val), _p(b), iters, _p(out))
    return out


def set_threads(t: int) -> None:
    """Host threads for the oracle's row loops (1 = sequential)."""
    _L().or_set_threads(int(t))


def get_threads() -> int:
    return int(_L().or_get_threads())


def lanczos_kappa(a, b, eps: float = 1e-10, maxit: int = 0, want_x: bool = False):
    """kappa-hat = lambda_max / lambda_min of the CG-Lanczos tridiagonal T_k
    of plain FP64 CG on (A, b) from 0, run to ||r|| <= eps ||b|| (maxit <= 0:
    10 n).  Returns (kappa_hat, lambda_min, lambda_max, k), and the CG iterate
    as a fifth item when want_x.  The extreme eigenvalues of T_k come from
    scipy's symmetric tridiagonal solver."""
    rp, col, val = _csr_arrays(a)
    b = np.ascontiguousarray(b, dtype=np.float64)
    m = int(maxit) if maxit > 0 else 10 * a.n
    al = np.zeros(m, dtype=np.float64)
    be = np.zeros(m, dtype=np.float64)
    x = np.zeros(a.n, dtype=np.float64) if want_x else None
    k = int(_L().or_cg_lanczos(a.n, _p(rp), _p(col), _p(val), _p(b), float(eps), m, _p(al), _p(be),
                               None if x is None else _p(x)))
    if k == 0:
        out = (float("nan"), float("nan"), float("nan"), 0)
        return out + (x,) if want_x else out
    al, be = al[:k], be[:k]
    diag = 1.0 / al
    diag[1:] += be[:-1] / al[:-1]
    off = np.sqrt(be[:-1]) / al[:-1]
    from scipy.linalg import eigvalsh_tridiagonal
    lam = eigvalsh_tridiagonal(diag, off)
    out = (float(lam[-1] / lam[0]), float(lam[0]), float(lam[-1]), k)
    return out + (x,) if want_x else out
