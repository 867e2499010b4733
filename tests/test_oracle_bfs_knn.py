"""Pins of the oracle's 2BFS pseudo-diameter, kNN selector and cost helpers
(no GPU): closed forms, brute force on small graphs, scipy/sklearn library
routines and the paper's printed training-size tables."""

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graph_csr(n, edges):
    ei = np.array([e[0] for e in edges], dtype=np.int64)
    ej = np.array([e[1] for e in edges], dtype=np.int64)
    return W.generators._graph_matrix(n, ei, ej, 1.1, 1.0, "g")


def _all_pairs(a):
    g = a.to_scipy().copy()
    g.setdiag(0)
    g.eliminate_zeros()
    g.data[:] = 1.0
    return shortest_path(g, unweighted=True, directed=False)


# ---------------------------------------------------------------- 2BFS --

@pytest.mark.parametrize("N", [2, 5, 64])
def test_grid2d_closed_form(N):
    ell, t, u, nc = oracle.pseudo_diameter(W.poisson2d(N))
    assert (ell, t, u, nc) == (2 * (N - 1), N * N - 1, 0, 1)


@pytest.mark.parametrize("N", [3, 7, 16])
def test_grid3d_closed_form(N):
    ell, t, u, nc = oracle.pseudo_diameter(W.poisson3d(N))
    assert (ell, t, u, nc) == (3 * (N - 1), N ** 3 - 1, 0, 1)


@pytest.mark.parametrize("n,w", [(1000, 8), (999, 8), (5001, 3), (17, 8)])
def test_banded_closed_form(n, w):
    ell, t, u, nc = oracle.pseudo_diameter(W.banded(n, w=w, seed=0))
    e = math.ceil((n - 1) / w)
    assert ell == e and nc == 1
    assert t == (e - 1) * w + 1   # smallest vertex at the largest distance from 0
    assert u == 0


def test_banded_one_million_closed_form():
    a = W.banded(1_000_000, w=8, seed=0)
    assert oracle.pseudo_diameter(a) == (125_000, 999_993, 0, 1)


def test_path_star_extended_star():
    assert oracle.pseudo_diameter(W.path(101))[0] == 100
    assert oracle.pseudo_diameter(W.star(1001)) == (2, 1, 2, 1)
    for lc, nc in [(5, 2), (10, 30), (1, 300), (4, 250)]:
        assert oracle.pseudo_diameter(W.extended_star(lc, nc))[0] == 2 * lc
    assert oracle.pseudo_diameter(W.extended_star(300, 1))[0] == 300


def test_diagonal_and_disjoint_union():
    d = W.CSR.from_scipy(sp.identity(7, format="csr") * 3.0)
    assert oracle.pseudo_diameter(d) == (0, 0, 0, 7)
    # union of a path of 10 (vertices 0..9) and a star of 5 (vertices 10..14)
    edges = [(i, i + 1) for i in range(9)] + [(10, j) for j in range(11, 15)]
    a = _graph_csr(15, edges)
    ell, t, u, nc = oracle.pseudo_diameter(a)
    assert (ell, nc) == (9, 2) and {t, u} == {0, 9}


def _random_tree(n, rng):
    return [(int(rng.integers(0, i)), i) for i in range(1, n)]


@pytest.mark.parametrize("seed", range(6))
def test_trees_double_sweep_is_exact_diameter(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 200))
    a = _graph_csr(n, _random_tree(n, rng))
    ap = _all_pairs(a)
    assert oracle.pseudo_diameter(a)[0] == int(ap.max())


@pytest.mark.parametrize("seed", range(8))
def test_general_graphs_bounded_by_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 200))
    edges = _random_tree(n, rng)
    extra = int(rng.integers(0, n))
    have = {(min(a, b), max(a, b)) for a, b in edges}
    while extra > 0:
        i, j = (int(v) for v in rng.integers(0, n, size=2))
        if i != j and (min(i, j), max(i, j)) not in have:
            have.add((min(i, j), max(i, j))); edges.append((i, j)); extra -= 1
    a = _graph_csr(n, edges)
    ap = _all_pairs(a)
    diam = int(ap.max())
    ell, t, u, nc = oracle.pseudo_diameter(a)
    assert math.ceil(diam / 2) <= ell <= diam
    # t is the smallest farthest vertex from 0, and ell = d(t, u) = ecc(t)
    d0 = ap[0]
    assert t == int(np.flatnonzero(d0 == d0.max())[0])
    assert ell == int(ap[t].max()) and u == int(np.flatnonzero(ap[t] == ap[t].max())[0])


@pytest.mark.parametrize("gen,src", [(lambda: W.er_laplacian(20000, 16, seed=1), 0),
                                     (lambda: W.varcoef3d(12, seed=0), 17),
                                     (lambda: W.banded(5000, 8, seed=0), 2500)])
def test_bfs_distances_equal_scipy(gen, src):
    a = gen()
    dist, ecc = oracle.bfs(a, src)
    g = a.to_scipy().copy(); g.setdiag(0); g.eliminate_zeros(); g.data[:] = 1.0
    ref = shortest_path(g, unweighted=True, directed=False, indices=[src])[0]
    ref = np.where(np.isinf(ref), -1, ref).astype(np.int32)
    assert np.array_equal(dist, ref) and ecc == ref.max()


# ----------------------------------------------------------------- kNN --

def test_knn_hand_examples():
    feat = np.array([[0, 0, 0, 0], [10, 0, 0, 0], [0, 10, 0, 0], [10, 10, 0, 0]], dtype=float)
    m = oracle.KnnModel.from_samples(feat, [2, 3, 4, 5], k=1, mask=15)
    # features 2 and 3 are constant -> normalised to 0
    t, sc, ex = oracle.knn_select(m, [9.0, 1.0, 0.0, 0.0])
    assert t == 3 and not ex
    assert sc[1] == pytest.approx(1.0 / math.hypot(0.1, 0.1))
    m3 = oracle.KnnModel.from_samples(feat, [2, 3, 3, 5], k=3, mask=15)
    # query (4,4) -> normalised (0.4, 0.4); distances: 0.566, 0.721, 0.721, 0.849
    t, sc, _ = oracle.knn_select(m3, [4.0, 4.0, 0.0, 0.0])
    d = [math.hypot(0.4, 0.4), math.hypot(0.6, 0.4), math.hypot(0.4, 0.6)]
    assert sc[0] == pytest.approx(1 / d[0]) and sc[1] == pytest.approx(1 / d[1] + 1 / d[2])
    assert t == 3


def test_knn_zero_distance_votes_by_count_and_ties_go_to_larger_eps1():
    feat = np.array([[1, 1, 1, 1], [1, 1, 1, 1], [2, 2, 2, 2], [3, 3, 3, 3]], dtype=float)
    m = oracle.KnnModel.from_samples(feat, [6, 4, 4, 4], k=3)
    t, sc, ex = oracle.knn_select(m, [1, 1, 1, 1])
    assert ex and sc[4] == 1.0 and sc[2] == 1.0 and t == 4   # 1-1 tie -> smaller t
    # equal distances: the earlier sample stays in the set (strict '<')
    m = oracle.KnnModel.from_samples(np.array([[0.0, 0, 0, 0], [2, 0, 0, 0], [4, 0, 0, 0], [2, 0, 0, 0]]),
                                     [2, 3, 4, 7], k=1)
    t, _, _ = oracle.knn_select(m, [2.0, 0, 0, 0])
    assert t == 3   # samples 1 and 3 both at distance 0; sample 1 entered first
    m = oracle.KnnModel.from_samples(np.array([[0.0, 0, 0, 0], [4, 0, 0, 0], [8, 0, 0, 0]]),
                                     [5, 2, 6], k=2)
    # query at 2: samples 0 and 1 both at 0.25, sample 2 at 0.75; 0 and 1 tie -> t = 2
    t, sc, _ = oracle.knn_select(m, [2.0, 0, 0, 0])
    assert sc[0] == sc[3] and t == 2


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 5), (2, 10), (3, 20)])
def test_knn_matches_sklearn_on_tie_free_data(seed, k):
    from sklearn.neighbors import KNeighborsClassifier
    rng = np.random.default_rng(seed)
    feat = rng.uniform(0, 1, size=(300, 4)) * np.array([1e5, 1e6, 500, 1.0])
    lab = rng.integers(2, 8, size=300)
    m = oracle.KnnModel.from_samples(feat, lab, k=k)
    norm = (feat - m.fmin) / (m.fmax - m.fmin)
    clf = KNeighborsClassifier(n_neighbors=k, weights="distance", algorithm="brute").fit(norm, lab)
    qs = rng.uniform(0, 1, size=(200, 4)) * np.array([1e5, 1e6, 500, 1.0])
    ref = clf.predict((qs - m.fmin) / (m.fmax - m.fmin))
    got = [oracle.knn_select(m, q)[0] for q in qs]
    assert list(ref) == got


def test_knn_feature_mask_three_d():
    rng = np.random.default_rng(5)
    feat = rng.uniform(0, 1, size=(50, 4))
    lab = rng.integers(2, 8, size=50)
    m4 = oracle.KnnModel.from_samples(feat, lab, k=1, mask=15)
    m3 = oracle.KnnModel.from_samples(feat, lab, k=1, mask=14)   # (m, ell, v) as in the paper
    q = feat[7].copy(); q[0] = 1e9
    assert oracle.knn_select(m3, q)[0] == lab[7]
    assert oracle.knn_select(m4, q)[2] is False


def test_model_file_roundtrip(tmp_path):
    rng = np.random.default_rng(1)
    m = oracle.KnnModel.from_samples(rng.uniform(0, 1, (20, 4)) * 1e3, rng.integers(2, 8, 20),
                                     k=3, omega=0.6)
    p = tmp_path / "m.txt"
    oracle.save_model(m, str(p))
    m2 = oracle.load_model(str(p))
    assert np.array_equal(m.feat, m2.feat) and np.array_equal(m.label, m2.label)
    assert np.array_equal(m.fmin, m2.fmin) and m2.k == 3 and m2.omega == 0.6


# ---------------------------------------------------------------- cost --

def test_training_size_tables_follow_eq26_k_dependence():
    """The printed N_S of the appendix scale as 1/(44 + 3k) (eqs. 24, 26): for
    k in {1, 5, 10, 20} one constant C reproduces every printed value after
    rounding.  The k = 15 column does not fit (a known misprint)."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "ns_training_sizes.txt"))
            if ln.strip() and not ln.startswith("#")]
    for r in rows:
        ns = dict(zip([1, 5, 10, 15, 20], (int(v) for v in r[1:])))
        lo, hi = -math.inf, math.inf
        for k in (1, 5, 10, 20):
            c = oracle.cost.knn_iteration_cycles(k)
            lo, hi = max(lo, (ns[k] - 0.5) * c), min(hi, (ns[k] + 0.5) * c)
        assert lo < hi
        c15 = oracle.cost.knn_iteration_cycles(15)
        assert not (lo / c15 - 0.5 <= ns[15] <= hi / c15 + 0.5)


def test_cost_model_formulas():
    assert oracle.cost.cost_I(12, 11, 1 / 3) == 15.0
    assert oracle.cost.efficiency(75.0, 100.0) == 25.0
    assert oracle.cost.overall_efficiency([10, 20], [20, 40]) == 50.0
    assert oracle.cost.bfs2_cycles(1000) == 2000
    # eq. (20): 2BFS below 1% of FP64 CG once k_CG >= 3 for c ~ 1
    n = m = 1000
    assert oracle.cost.bfs2_cycles(m) < 0.01 * oracle.cost.cg_dp_cycles(n, m, 3)
