"""Pins of the oracle's multi-start 2BFS and effective diameter against
brute-force all-pairs distances (scipy) -- facts that do not come from the
oracle itself:
  * with every vertex as a start, max_s l(t_s, u_s) is the exact diameter
    (l(t_s, u_s) >= d(s, t_s) = ecc(s), and max_s ecc(s) is the diameter);
  * with every vertex as a start, the effective diameter is the q-quantile
    rule applied to the all-pairs distance distribution;
  * on trees a single 2BFS is already exact;
  * pdiam <= pdiam_multi <= diameter for any set of starts."""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import workloads as W
from workloads import paper_family as PF


def _allpairs(a):
    g = a.to_scipy().copy()
    g.setdiag(0)
    g.eliminate_zeros()
    g.data[:] = 1.0
    return csg.shortest_path(g, unweighted=True, directed=False)


def _quantile_rule(dists, q):
    d = dists[np.isfinite(dists) & (dists > 0)].astype(np.int64)
    if d.size == 0:
        return 0, 0
    h = np.bincount(d)
    cum = np.cumsum(h)
    for k in range(1, h.size):
        if cum[k] >= q * d.size:
            return k, d.size
    raise AssertionError


def _graphs():
    yield "grid", W.poisson2d(9)
    yield "path", W.path(40)
    yield "xstar", W.extended_star(5, 7, extra_edges=4, seed=2)
    yield "random", PF.random_sparse(120, 0.5, 1.1, seed=3)
    yield "band_sparse", PF.random_banded(150, 5, 0.4, 1.1, seed=4)   # disconnected, isolated vertices
    yield "er", W.er_laplacian(150, 4, seed=5)
    yield "union", W.CSR.from_scipy(sp.block_diag([W.path(20).to_scipy(), W.poisson2d(5).to_scipy()]).tocsr())


@pytest.mark.parametrize("name,a", list(_graphs()))
@pytest.mark.parametrize("q", [0.5, 0.9, 1.0])
def test_all_starts_give_exact_diameter_and_quantile(name, a, q):
    D = _allpairs(a)
    diam = int(np.max(D[np.isfinite(D)]))
    pd, pdm, eff, pairs, best = oracle.diameter_multi(a, list(range(a.n)), q)
    assert pdm == diam
    assert pd <= pdm
    e, np_ = _quantile_rule(D, q)
    assert (eff, pairs) == (e, np_)


@pytest.mark.parametrize("name,a", list(_graphs()))
def test_subsets_are_bounded(name, a):
    D = _allpairs(a)
    diam = int(np.max(D[np.isfinite(D)]))
    rng = np.random.default_rng(9)
    for _ in range(5):
        starts = rng.choice(a.n, size=min(6, a.n), replace=False).tolist()
        pd, pdm, eff, pairs, best = oracle.diameter_multi(a, starts, 0.9)
        assert pd <= pdm <= diam
        e, np_ = _quantile_rule(D[starts, :], 0.9)
        assert (eff, pairs) == (e, np_)
        assert (best == -1) == (pdm == pd)


def test_tree_single_2bfs_is_exact():
    for seed in range(4):
        rng = np.random.default_rng(seed)
        p, c = PF.random_tree_edges(200, rng)
        t = sp.coo_matrix((np.ones(p.size), (p, c)), shape=(200, 200))
        a = W.CSR.from_scipy(t + t.T + sp.identity(200))
        D = _allpairs(a)
        pd, pdm, *_ = oracle.diameter_multi(a, [7, 50], 0.9)
        assert pd == pdm == int(D.max())


def test_q_one_is_largest_start_eccentricity():
    a = PF.random_sparse(150, 1.0, 3.0, seed=8)
    starts = [3, 17, 99]
    D = _allpairs(a)
    _, _, eff, _, _ = oracle.diameter_multi(a, starts, 1.0)
    assert eff == int(D[starts].max())


def test_edge_cases():
    a = W.poisson2d(6)
    pd, pdm, eff, pairs, best = oracle.diameter_multi(a, [], 0.9)
    assert (pdm, eff, pairs, best) == (pd, 0, 0, -1)
    # an isolated start contributes no pair
    b = W.CSR.from_scipy(sp.block_diag([W.path(5).to_scipy(), sp.csr_matrix(np.array([[2.0]]))]).tocsr())
    assert oracle.diameter_multi(b, [5], 0.9)[2:4] == (0, 0)
    with pytest.raises(ValueError):
        oracle.diameter_multi(a, [36], 0.9)
    with pytest.raises(ValueError):
        oracle.diameter_multi(a, [0], 0.0)
