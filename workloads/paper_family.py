"""Seeded generators of the paper's three experimental matrix families.

Section "Samples used in computational experiments" and the appendix on
sample generation describe them; every matrix is built from the adjacency
matrix of an undirected graph, with diagonal a_ii = mu * sum_{j != i} |a_ij|
(strict diagonal dominance, hence SPD), mu in {1.1, 3, 10}:

  * perturbed extended stars: a centre joined to nc rays of lc vertices
    (n = 1 + nc*lc, the (lc, nc) pairs of the appendix tables) plus xi
    distinct random edges, xi uniform in [0, 0.1 n); off-diagonal entries 1.
  * random sparse: a random tree on n vertices plus floor(c n) distinct random
    edges, c in {0.1, 0.5, 1, 2, 3, 5, 7, 10}; entries by Algorithm III.
  * random banded: every pair with 1 <= |i - j| <= w present independently
    with probability p in {0.4, 0.6, 0.8}, full bandwidth b = 2w + 1 odd in
    {3, ..., b_max(n)}; entries by Algorithm III.

Algorithm III (appendix) gives each edge (i < j, in row-major order) the value
+-U(0, 3) or +-U(7, 10): xi_d ~ U(0,1) picks the range (> 0.5: [0, 3]),
xi_s ~ U(0,1) the sign (> 0.5: +), and the magnitude is drawn in that range;
a_ji = a_ij.  The three uniforms of an edge are drawn in that order.

Readings where the appendix leaves a choice (all stated again where used):
  * the random tree is a random recursive tree: vertex i >= 1 joins a
    uniformly drawn earlier vertex;
  * the general sample sizes of the appendix factor as (lc, nc) pairs x 100
    x 3 mu values (stars), 8 c values x 3 mu values x 200 (random) and 3 p
    values x odd b values x 20 x 2 mu values (banded: mu in {1.1, 3});
  * right-hand sides: x ~ U(1, 2), b = A x.

The module draws inputs only; none of the method's arithmetic is here.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .generators import CSR, _coo_to_csr, extended_star

MU = (1.1, 3.0, 10.0)
MU_BANDED = (1.1, 3.0)
RANDOM_C = (0.1, 0.5, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0)
BANDED_P = (0.4, 0.6, 0.8)

# (lc, nc) of the extended stars (appendix tables for n = 301, 501, 1001)
STAR_LC_NC = {
    301: ((1, 300), (2, 150), (5, 60), (10, 30), (15, 20), (20, 15), (30, 10), (60, 5), (150, 2), (300, 1)),
    501: ((1, 500), (2, 250), (4, 125), (5, 100), (10, 50), (20, 25), (25, 20), (50, 10), (100, 5),
          (125, 4), (250, 2), (500, 1)),
    1001: ((1, 1000), (2, 500), (4, 250), (5, 200), (8, 125), (10, 100), (20, 50), (25, 40), (40, 25),
           (50, 20), (100, 10), (125, 8), (200, 5), (250, 4), (500, 2), (1000, 1)),
}
# largest full bandwidth for each banded matrix size
BANDED_B_MAX = {300: 29, 500: 51, 1000: 101}

ALG3_RANGES = ((0.0, 3.0), (7.0, 10.0))


def algorithm3_values(n_edges: int, rng, ranges=ALG3_RANGES) -> np.ndarray:
    """Algorithm III values for n_edges edges in row-major edge order."""
    (a1, b1), (a2, b2) = ranges
    u = rng.random((n_edges, 3))            # xi_d, xi_s, magnitude draw per edge
    lo = np.where(u[:, 0] > 0.5, a1, a2)
    hi = np.where(u[:, 0] > 0.5, b1, b2)
    mag = lo + (hi - lo) * u[:, 2]
    return np.where(u[:, 1] > 0.5, mag, -mag)


def _dominant(n, ei, ej, w, mu, name) -> CSR:
    """a_ij = a_ji = w for each edge, a_ii = mu * sum_{j != i} |a_ij|."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    aw = np.abs(w)
    rs = np.bincount(ei, weights=aw, minlength=n) + np.bincount(ej, weights=aw, minlength=n)
    i = np.arange(n, dtype=np.int64)
    rows = np.concatenate([ei, ej, i])
    cols = np.concatenate([ej, ei, i])
    vals = np.concatenate([w, w, mu * rs])
    keep = vals != 0.0
    return _coo_to_csr(n, rows[keep], cols[keep], vals[keep], name=name)


def _sorted_edges(ei, ej):
    """Edges as (i < j), sorted row-major (the order Algorithm III visits them)."""
    lo = np.minimum(ei, ej)
    hi = np.maximum(ei, ej)
    order = np.lexsort((hi, lo))
    return lo[order], hi[order]


def _add_random_edges(n: int, have: set, count: int, rng):
    """`count` distinct unordered pairs {i, j}, i != j, not in `have` (keys i*n+j)."""
    add_i, add_j = [], []
    while len(add_i) < count:
        need = count - len(add_i)
        draw = rng.integers(0, n, size=(max(2 * need, 16), 2))
        for a, b in draw.tolist():
            if a == b:
                continue
            lo, hi = (a, b) if a < b else (b, a)
            key = lo * n + hi
            if key in have:
                continue
            have.add(key)
            add_i.append(lo)
            add_j.append(hi)
            if len(add_i) == count:
                break
    return np.array(add_i, dtype=np.int64), np.array(add_j, dtype=np.int64)


def perturbed_extended_star(lc: int, nc: int, mu: float, seed: int) -> CSR:
    """Extended star (lc, nc) plus xi ~ U{0, ..., ceil(0.1 n) - 1} random edges; entries 1."""
    n = 1 + nc * lc
    rng = np.random.default_rng(seed)
    xi = int(rng.integers(0, max(1, math.ceil(0.1 * n))))
    return extended_star(lc, nc, extra_edges=xi, seed=seed + 1, mu=mu, weight=1.0)


def random_tree_edges(n: int, rng):
    """Random recursive tree: vertex i >= 1 joins a uniform earlier vertex."""
    if n <= 1:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    child = np.arange(1, n, dtype=np.int64)
    parent = np.floor(rng.random(n - 1) * child).astype(np.int64)
    return parent, child


def random_sparse(n: int, c: float, mu: float, seed: int) -> CSR:
    """Random tree plus floor(c n) distinct random edges; Algorithm III values."""
    rng = np.random.default_rng(seed)
    ti, tj = random_tree_edges(n, rng)
    have = set((np.minimum(ti, tj) * n + np.maximum(ti, tj)).tolist())
    ai, aj = _add_random_edges(n, have, int(math.floor(c * n)), rng)
    ei, ej = _sorted_edges(np.concatenate([ti, ai]), np.concatenate([tj, aj]))
    w = algorithm3_values(ei.size, rng)
    return _dominant(n, ei, ej, w, mu, name=f"rand_{n}_c{c:g}_mu{mu:g}_s{seed}")


def random_banded(n: int, b: int, p: float, mu: float, seed: int) -> CSR:
    """Pairs with 1 <= j - i <= (b - 1) / 2 present with probability p; Algorithm III values."""
    if b < 3 or b % 2 == 0:
        raise ValueError("full bandwidth b must be odd and >= 3")
    w = (b - 1) // 2
    rng = np.random.default_rng(seed)
    ii, jj = [], []
    for d in range(1, w + 1):
        i = np.arange(0, n - d, dtype=np.int64)
        ii.append(i)
        jj.append(i + d)
    ei = np.concatenate(ii)
    ej = np.concatenate(jj)
    ei, ej = _sorted_edges(ei, ej)
    keep = rng.random(ei.size) < p
    ei, ej = ei[keep], ej[keep]
    vals = algorithm3_values(ei.size, rng)
    return _dominant(n, ei, ej, vals, mu, name=f"band_{n}_b{b}_p{p:g}_mu{mu:g}_s{seed}")


def sample_specs(family: str, n: int, scale: float = 1.0, seed: int = 0):
    """The general sample S0 of one family and size as a list of generator
    specs (family, params, seed); `scale` < 1 keeps that fraction of the
    matrices of every parameter combination (at least one)."""
    specs = []
    s = seed * 1_000_003
    if family == "star":
        pairs = STAR_LC_NC[n]
        per = max(1, int(round(100 * scale)))
        for lc, nc in pairs:
            for mu in MU:
                for r in range(per):
                    s += 1
                    specs.append(("star", (lc, nc, mu), s))
    elif family == "random":
        per = max(1, int(round(200 * scale)))
        for c in RANDOM_C:
            for mu in MU:
                for r in range(per):
                    s += 1
                    specs.append(("random", (n, c, mu), s))
    elif family == "banded":
        per = max(1, int(round(20 * scale)))
        for p in BANDED_P:
            for b in range(3, BANDED_B_MAX[n] + 1, 2):
                for mu in MU_BANDED:
                    for r in range(per):
                        s += 1
                        specs.append(("banded", (n, b, p, mu), s))
    else:
        raise ValueError(f"unknown family {family!r}")
    return specs


def make(spec) -> CSR:
    family, prm, seed = spec
    if family == "star":
        lc, nc, mu = prm
        return perturbed_extended_star(lc, nc, mu, seed)
    if family == "random":
        n, c, mu = prm
        return random_sparse(n, c, mu, seed)
    if family == "banded":
        n, b, p, mu = prm
        return random_banded(n, b, p, mu, seed)
    raise ValueError(f"unknown family {family!r}")


def paper_rhs(a: CSR, seed: int):
    """x ~ U(1, 2), b = A x (FP64, on the host)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(1.0, 2.0, size=a.n)
    b = a.to_scipy() @ x
    return x, np.ascontiguousarray(b, dtype=np.float64)
