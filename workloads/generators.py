"""Seeded generators for sparse SPD systems in CSR form.

Every generator is deterministic for a given seed (numpy PCG64 via
``default_rng``), orders unknowns lexicographically and returns CSR with
sorted column indices, no duplicates and no stored zeros.  Values are FP64.

Families:
  * ``poisson2d``   5-point Laplacian on an N x N grid (4 / -1).
  * ``poisson3d``   7-point Laplacian on an N^3 grid (6 / -1).
  * ``varcoef3d``   7-point variable-coefficient diffusion on an N^3 grid; every
                    cell face (boundary faces included, Dirichlet ghost = 0) gets
                    k_f = 10**U(0,3); A_pq = -k_f, A_pp = sum of the cell's six
                    face coefficients.
  * ``banded``      a_ij = a_ji ~ U[-1,0) for 1 <= |i-j| <= w,
                    a_ii = sum_j |a_ij| + 1e-4.
  * ``er_laplacian`` G(n, M) with M distinct uniform unordered pairs and no
                    self-loops; L = D - Adj + shift * I.
  * ``star`` / ``path`` / ``extended_star``  graph matrices in the style of the
                    paper's experiment section: off-diagonal entries equal to the
                    adjacency entries and a_ii = mu * sum_{j != i} |a_ij|.

``rhs`` draws x* and forms b = A x* once, on the host, in FP64.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: 0-based, sorted columns, int64 row pointers."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(a, name: str = "") -> "CSR":
        a = sp.csr_matrix(a)
        a.sum_duplicates()
        a.sort_indices()
        a.eliminate_zeros()
        return CSR(
            n=a.shape[0],
            row_ptr=np.ascontiguousarray(a.indptr, dtype=np.int64),
            col=np.ascontiguousarray(a.indices, dtype=np.int32),
            val=np.ascontiguousarray(a.data, dtype=np.float64),
            name=name,
        )

    def bandwidth(self) -> int:
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        if rows.size == 0:
            return 0
        return int(np.max(np.abs(rows - self.col.astype(np.int64))))


def _coo_to_csr(n, rows, cols, vals, name):
    a = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    return CSR.from_scipy(a, name=name)


def poisson2d(N: int) -> CSR:
    """5-point Laplacian, n = N^2, m = 5N^2 - 4N, values 4 / -1."""
    t = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    eye = sp.identity(N)
    a = sp.kron(eye, t) + sp.kron(t, eye)
    return CSR.from_scipy(a, name=f"poisson2d_{N}")


def poisson3d(N: int) -> CSR:
    """7-point Laplacian, n = N^3, values 6 / -1."""
    t = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    eye = sp.identity(N)
    a = sp.kron(sp.kron(eye, eye), t) + sp.kron(sp.kron(eye, t), eye) + sp.kron(sp.kron(t, eye), eye)
    return CSR.from_scipy(a, name=f"poisson3d_{N}")


def varcoef3d(N: int, seed: int = 0, decades: float = 3.0) -> CSR:
    """7-point variable-coefficient diffusion on an N^3 grid.

    Cell p = (k*N + j)*N + i.  Face coefficients are drawn in the order x-faces
    (shape N,N,N+1), y-faces (N,N+1,N), z-faces (N+1,N,N), each as
    10**U(0, decades).
    """
    rng = np.random.default_rng(seed)
    fx = 10.0 ** rng.uniform(0.0, decades, size=(N, N, N + 1))
    fy = 10.0 ** rng.uniform(0.0, decades, size=(N, N + 1, N))
    fz = 10.0 ** rng.uniform(0.0, decades, size=(N + 1, N, N))
    diag = fx[:, :, :-1] + fx[:, :, 1:] + fy[:, :-1, :] + fy[:, 1:, :] + fz[:-1, :, :] + fz[1:, :, :]
    idx = np.arange(N * N * N, dtype=np.int64).reshape(N, N, N)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # x neighbours: (k,j,i-1) - (k,j,i), i = 1..N-1, coefficient fx[k,j,i]
    a, b, c = idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel(), -fx[:, :, 1:-1].ravel()
    rows += [a, b]; cols += [b, a]; vals += [c, c]
    a, b, c = idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel(), -fy[:, 1:-1, :].ravel()
    rows += [a, b]; cols += [b, a]; vals += [c, c]
    a, b, c = idx[:-1, :, :].ravel(), idx[1:, :, :].ravel(), -fz[1:-1, :, :].ravel()
    rows += [a, b]; cols += [b, a]; vals += [c, c]
    return _coo_to_csr(N ** 3, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                       name=f"varcoef3d_{N}_s{seed}")


def banded(n: int, w: int = 8, seed: int = 0, shift: float = 1e-4) -> CSR:
    """Full band of half-width w: a_ij = a_ji ~ U[-1,0), a_ii = row |sum| + shift.

    Off-diagonals are drawn diagonal by diagonal, d = 1..w, each as n-d values.
    """
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    absrow = np.zeros(n)
    for d in range(1, w + 1):
        if n - d <= 0:
            break
        v = rng.uniform(-1.0, 0.0, size=n - d)
        # U[-1,0) from uniform(-1,0) never returns 0 exactly except with prob 0;
        # guard anyway so that no explicit zero is stored.
        v[v == 0.0] = -0.5
        i = np.arange(n - d, dtype=np.int64)
        rows += [i, i + d]; cols += [i + d, i]; vals += [v, v]
        absrow[: n - d] += -v
        absrow[d:] += -v
    i = np.arange(n, dtype=np.int64)
    rows.append(i); cols.append(i); vals.append(absrow + shift)
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                       name=f"banded_{n}_w{w}_s{seed}")


def _distinct_pairs(n: int, m_edges: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """First m_edges distinct unordered pairs {i,j}, i != j, in draw order."""
    keys = np.empty(0, dtype=np.int64)
    need = m_edges
    while True:
        draw = max(int(need * 1.1) + 16, 1024)
        ij = rng.integers(0, n, size=(draw, 2), dtype=np.int64)
        ok = ij[:, 0] != ij[:, 1]
        ij = ij[ok]
        lo = np.minimum(ij[:, 0], ij[:, 1]); hi = np.maximum(ij[:, 0], ij[:, 1])
        keys = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(keys, return_index=True)
        if first.size >= m_edges:
            first.sort()
            keys = keys[first[:m_edges]]
            break
        first.sort()
        keys = keys[first]
        need = m_edges - keys.size
    return keys // n, keys % n


def er_laplacian(n: int, avg_degree: int = 16, seed: int = 0, shift: float = 1e-3) -> CSR:
    """Erdos-Renyi G(n, M) with M = n*avg_degree/2 edges, L = D - Adj + shift*I."""
    rng = np.random.default_rng(seed)
    m_edges = n * avg_degree // 2
    a, b = _distinct_pairs(n, m_edges, rng)
    deg = np.bincount(a, minlength=n) + np.bincount(b, minlength=n)
    i = np.arange(n, dtype=np.int64)
    rows = np.concatenate([a, b, i]); cols = np.concatenate([b, a, i])
    vals = np.concatenate([-np.ones(m_edges), -np.ones(m_edges), deg.astype(np.float64) + shift])
    return _coo_to_csr(n, rows, cols, vals, name=f"er_{n}_d{avg_degree}_s{seed}")


def _graph_matrix(n, ei, ej, mu, weight, name):
    """Symmetric matrix from an edge list: a_ij = weight, a_ii = mu * sum |a_ij|."""
    ei = np.asarray(ei, dtype=np.int64); ej = np.asarray(ej, dtype=np.int64)
    w = np.full(ei.size, float(weight))
    deg = np.bincount(ei, minlength=n) + np.bincount(ej, minlength=n)
    i = np.arange(n, dtype=np.int64)
    diag = mu * abs(weight) * deg.astype(np.float64)
    rows = np.concatenate([ei, ej, i]); cols = np.concatenate([ej, ei, i])
    vals = np.concatenate([w, w, diag])
    keep = vals != 0.0
    return _coo_to_csr(n, rows[keep], cols[keep], vals[keep], name=name)


def star(n: int, mu: float = 1.1, weight: float = 1.0) -> CSR:
    """Star graph: centre 0 joined to 1..n-1."""
    leaves = np.arange(1, n)
    return _graph_matrix(n, np.zeros(n - 1, dtype=np.int64), leaves, mu, weight, f"star_{n}")


def path(n: int, mu: float = 1.1, weight: float = 1.0) -> CSR:
    """Path graph 0-1-...-(n-1)."""
    i = np.arange(n - 1)
    return _graph_matrix(n, i, i + 1, mu, weight, f"path_{n}")


def extended_star(lc: int, nc: int, extra_edges: int = 0, seed: int = 0, mu: float = 1.1,
                  weight: float = 1.0) -> CSR:
    """Centre vertex 0 with nc rays of lc vertices each (n = 1 + nc*lc), plus
    ``extra_edges`` distinct random edges not already present."""
    n = 1 + nc * lc
    ei, ej = [], []
    for r in range(nc):
        first = 1 + r * lc
        ei.append(0); ej.append(first)
        for q in range(lc - 1):
            ei.append(first + q); ej.append(first + q + 1)
    ei = np.array(ei, dtype=np.int64); ej = np.array(ej, dtype=np.int64)
    if extra_edges > 0:
        rng = np.random.default_rng(seed)
        existing = set((min(a, b) * n + max(a, b)) for a, b in zip(ei.tolist(), ej.tolist()))
        add = []
        while len(add) < extra_edges:
            a, b = rng.integers(0, n, size=2)
            if a == b:
                continue
            key = int(min(a, b)) * n + int(max(a, b))
            if key in existing:
                continue
            existing.add(key)
            add.append((int(min(a, b)), int(max(a, b))))
        ei = np.concatenate([ei, np.array([p[0] for p in add], dtype=np.int64)])
        ej = np.concatenate([ej, np.array([p[1] for p in add], dtype=np.int64)])
    return _graph_matrix(n, ei, ej, mu, weight, f"xstar_{lc}x{nc}_e{extra_edges}_s{seed}")


def random_spd_dense(n: int, seed: int = 0, eigs=None):
    """Dense SPD matrix Q diag(eigs) Q^T (symmetrised) and its CSR form."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    if eigs is None:
        eigs = rng.uniform(1.0, 10.0, size=n)
    a = (q * np.asarray(eigs, dtype=np.float64)) @ q.T
    a = 0.5 * (a + a.T)
    return a, CSR.from_scipy(sp.csr_matrix(a), name=f"dense_spd_{n}_s{seed}")


def rhs(a: CSR, seed: int = 0, low: float = -1.0, high: float = 1.0):
    """x* ~ U[low, high) and b = A x* (FP64, computed once on the host)."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(low, high, size=a.n)
    b = a.to_scipy() @ xs
    return xs, np.ascontiguousarray(b, dtype=np.float64)


FAMILIES = ("lap2d", "lap3d", "banded", "er")


def smooth_rhs(a: CSR):
    """x*_i = sin(pi (i + 1) / (n + 1)) (the lowest mode of a 1D chain) and
    b = A x* in FP64.  On a weakly shifted band this makes ||b|| far smaller
    than ||A|| ||x*||, so the recursive CG residual drifts measurably from
    the true one before it reaches a tight tolerance."""
    i = np.arange(a.n, dtype=np.float64)
    x = np.sin(np.pi * (i + 1.0) / (a.n + 1.0))
    return x, a.to_scipy() @ x


def family_matrix(family: str, n_target: int, seed: int) -> CSR:
    """One matrix of a family at roughly n_target unknowns (grids round to N^2 / N^3)."""
    if family == "lap2d":
        N = max(2, int(round(math.sqrt(n_target))))
        return poisson2d(N)
    if family == "lap3d":
        N = max(2, int(round(n_target ** (1.0 / 3.0))))
        return varcoef3d(N, seed=seed)
    if family == "banded":
        return banded(max(16, n_target), w=8, seed=seed)
    if family == "er":
        return er_laplacian(max(64, n_target), avg_degree=16, seed=seed)
    raise ValueError(f"unknown family {family!r}")
