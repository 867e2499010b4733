"""GPU parity of the batched engine (mpcg_batch_* through the C ABI) against
the CPU oracle, plus the batch-specific properties.

Bars (as for single solves):
  * every system: status OK, final true relative residual <= eps2, iteration
    counts per phase within max(1, ceil(5%)) of the oracle's, relative
    difference of x <= 1e-8;
  * Algorithm II systems: 2BFS pseudo-diameter, t, u and component count
    bit-exact with the oracle, v within 1e-9, the kNN class equal to the
    oracle selector's on the GPU's features;
  * a system gives the same bits (x, counts, eps1) alone and in any mix.
"""

import math
import os
import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TEST_MODEL = os.path.join(GOLDEN, "knn_model_test.txt")
EPS2 = 1e-10


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


@pytest.fixture(scope="module")
def engine(torch_mod):
    from paper_2412_08059_amd import BatchSolver
    e = BatchSolver(600_000, 6_000_000, 64, model=TEST_MODEL)
    yield e
    e.close()


def band_ok(n_gpu, n_or):
    return abs(n_gpu - n_or) <= max(1, math.ceil(0.05 * n_or))


def _disconnected():
    a = W.poisson2d(20).to_scipy()
    b = W.banded(700, 3, seed=4).to_scipy()
    return W.CSR.from_scipy(sp.block_diag([a, sp.csr_matrix(np.array([[2.0]])), b]).tocsr())


MIX = [
    ("poisson2d_40_e4", lambda: W.poisson2d(40), 1e-4),
    ("poisson2d_64_auto", lambda: W.poisson2d(64), 0.0),
    ("varcoef3d_16_none", lambda: W.varcoef3d(16, seed=2), -1.0),
    ("varcoef3d_20_auto", lambda: W.varcoef3d(20, seed=1), 0.0),
    ("banded_6000_e6", lambda: W.banded(6000, 8, seed=1), 1e-6),
    ("banded_3000_auto", lambda: W.banded(3000, 8, seed=5), 0.0),
    ("er_8000_e3", lambda: W.er_laplacian(8000, 16, seed=2), 1e-3),
    ("er_5000_auto", lambda: W.er_laplacian(5000, 16, seed=6), 0.0),
    ("star_1001_e2", lambda: W.star(1001, mu=1.1), 1e-2),
    ("disconnected_auto", _disconnected, 0.0),
    ("one_by_one_e4", lambda: W.CSR.from_scipy(sp.csr_matrix(np.array([[3.0]]))), 1e-4),
]


def _make(torch, name, gen, eps1, seed):
    from paper_2412_08059_amd import DeviceCSR
    a = gen()
    _, b = W.rhs(a, seed=seed)
    B = torch.from_numpy(b).cuda()
    X = torch.full((a.n,), float("nan"), dtype=torch.float64, device="cuda")
    return a, b, (DeviceCSR.from_host(a), B, X, eps1, EPS2)


def _check_against_oracle(a, b, eps1, st, x, model):
    r = oracle.solve(a, b, eps1, EPS2, model=model if eps1 == 0.0 else None)
    assert st.status == 0 and r.status == 0, (st.status, r.status)
    assert st.relres_final_true <= EPS2
    assert band_ok(st.n1, r.n1), (st.n1, r.n1)
    assert band_ok(st.n2, r.n2), (st.n2, r.n2)
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - r.x) / np.linalg.norm(r.x) <= 1e-8
    if eps1 == 0.0:
        f = st.feat
        assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == oracle.pseudo_diameter(a)
        assert f.k0_used == r.k0_used
        assert abs(f.v - r.v) <= 1e-9 * max(1.0, abs(r.v))
        t_or, _, _ = oracle.knn_select(model, [f.n, f.m, f.pdiam, f.v])
        assert st.eps1_class == t_or == r.eps1_class
    elif eps1 == -1.0:
        assert st.n1 == 0 and st.eps1_class == -1
    return r


def test_batch_mix_matches_oracle(engine, torch_mod):
    model = oracle.load_model(TEST_MODEL)
    items = [(_make(torch_mod, nm, g, e, seed=i), nm, e) for i, (nm, g, e) in enumerate(MIX)]
    print(f"batch mix of {len(items)} systems", flush=True)
    ids = engine.submit([it[0][2] for it in items])
    got = engine.wait_all(ids, timeout_s=120)
    for rid, ((a, b, _), nm, e) in zip(ids, items):
        st, x = got[rid]
        print(f"  {nm}: status={st.status} n1={st.n1} n2={st.n2} cls={st.eps1_class}", flush=True)
        _check_against_oracle(a, b, e, st, x, model)


@pytest.mark.parametrize("runahead,band", [(1, 0), (2, 0), (2, 1), (0, 1)])
def test_batch_run_ahead_restarts_from_the_crossing(torch_mod, runahead, band):
    """Features that arrive long after the FP32 phase has passed every
    candidate eps1: a path-like band (tridiagonal, mu = 1.1, n = 50000) has a
    2BFS of 2 x 49999 levels while its CG crosses 1e-7 within a few dozen
    iterations (with the level kernels; the band sweeps take a few ms).
    Whether the system runs ahead (copies of x~ at each crossing, a
    speculative FP64 phase: runahead 1, or 0 with few systems listed) or
    waits at its first crossing (runahead 2), the FP64 restart
    must start from the state the sequential Algorithm II stops in, so the
    result matches the oracle's Algorithm II."""
    from paper_2412_08059_amd import BatchSolver
    from workloads import paper_family as PF
    model = oracle.load_model(TEST_MODEL)
    a, b, req = _make(torch_mod, "band_path_auto", lambda: PF.random_banded(50_000, 3, 1.0, 1.1, seed=3), 0.0,
                      seed=17)
    eng = BatchSolver(100_000, 1_000_000, 4, model=TEST_MODEL,
                      tuning={"batch_runahead": runahead, "batch_bfs_band": band})
    try:
        (rid,) = eng.submit([req])
        st, x = eng.wait_all([rid], timeout_s=120)[rid]
    finally:
        eng.close()
    print(f"  band_path_auto runahead={runahead} band={band}: status={st.status} n1={st.n1} n2={st.n2} "
          f"cls={st.eps1_class} pdiam={st.feat.pdiam} t_feat={st.t_feat_ms:.1f} ms", flush=True)
    assert st.feat.pdiam == 49_999
    _check_against_oracle(a, b, 0.0, st, x, model)


def test_batch_alone_equals_in_mix_bitwise(engine, torch_mod):
    """A system's result does not depend on the other systems in the batch."""
    probe = [("varcoef3d_18_auto", lambda: W.varcoef3d(18, seed=3), 0.0),
             ("banded_4000_e5", lambda: W.banded(4000, 8, seed=8), 1e-5),
             ("er_6000_none", lambda: W.er_laplacian(6000, 16, seed=9), -1.0)]
    alone = {}
    for nm, g, e in probe:
        a, b, req = _make(torch_mod, nm, g, e, seed=21)
        (rid,) = engine.submit([req])
        st, x = engine.wait_all([rid], timeout_s=60)[rid]
        assert st.status == 0
        alone[nm] = (st.n1, st.n2, st.eps1_class, x.cpu().numpy().copy())
    # the same systems among others, submitted in two waves while the first runs
    others = [_make(torch_mod, f"fill{i}", lambda i=i: W.poisson2d(30 + 3 * i), 1e-3 if i % 2 else 0.0, seed=40 + i)
              for i in range(6)]
    mix_reqs = [others[0][2], others[1][2]]
    probes = {nm: _make(torch_mod, nm, g, e, seed=21) for nm, g, e in probe}
    ids_a = engine.submit(mix_reqs + [probes[probe[0][0]][2]])
    time.sleep(0.002)
    ids_b = engine.submit([o[2] for o in others[2:]] + [probes[nm][2] for nm, _, _ in probe[1:]])
    got = engine.wait_all(ids_a + ids_b, timeout_s=120)
    pid = {probe[0][0]: ids_a[-1], probe[1][0]: ids_b[-2], probe[2][0]: ids_b[-1]}
    for nm, rid in pid.items():
        st, x = got[rid]
        n1, n2, cls, xa = alone[nm]
        assert (st.n1, st.n2, st.eps1_class) == (n1, n2, cls), nm
        assert np.array_equal(x.cpu().numpy().view(np.uint64), xa.view(np.uint64)), nm


def test_batch_edge_cases(engine, torch_mod):
    from paper_2412_08059_amd import DeviceCSR, capi
    torch = torch_mod
    # zero right-hand side: x = 0, no iterations
    a = W.poisson2d(12)
    A = DeviceCSR.from_host(a)
    Z = torch.zeros(a.n, dtype=torch.float64, device="cuda")
    X0 = torch.full((a.n,), 5.0, dtype=torch.float64, device="cuda")
    # malformed matrix: a column index out of range -> EINVAL for that request only
    bad = W.poisson2d(10)
    col = bad.col.copy()
    col[7] = bad.n + 3
    Abad = DeviceCSR(torch.from_numpy(bad.row_ptr.astype(np.int32)).cuda(), torch.from_numpy(col).cuda(),
                     torch.from_numpy(bad.val).cuda(), bad.n)
    _, bb = W.rhs(bad, seed=1)
    Bb = torch.from_numpy(bb).cuda()
    Xb = torch.empty(bad.n, dtype=torch.float64, device="cuda")
    good = _make(torch, "good", lambda: W.poisson2d(24), 1e-4, seed=3)
    print("batch edge cases", flush=True)
    ids = engine.submit([(A, Z, X0, 1e-4, EPS2), (Abad, Bb, Xb, 1e-4, EPS2), good[2]])
    got = engine.wait_all(ids, timeout_s=60)
    st0, x0 = got[ids[0]]
    assert st0.status == 0 and st0.n1 == 0 and st0.n2 == 0
    assert np.all(x0.cpu().numpy() == 0.0)
    assert got[ids[1]][0].status == capi.MPCG_EINVAL
    assert got[ids[2]][0].status == 0 and got[ids[2]][0].relres_final_true <= EPS2
    # larger than the whole arena: rejected at submission, nothing queued
    big = W.poisson2d(800)   # 640k rows > 600k
    with pytest.raises(Exception):
        engine.submit([(DeviceCSR.from_host(big), torch.zeros(big.n, dtype=torch.float64, device="cuda"),
                        torch.empty(big.n, dtype=torch.float64, device="cuda"), 1e-4, EPS2)])
    # bad tolerance: rejected at submission
    with pytest.raises(Exception):
        engine.submit([(A, Z, X0, 1e-4, -1.0)])


def test_batch_cancel(engine, torch_mod):
    from paper_2412_08059_amd import capi
    slow = _make(torch_mod, "slow", lambda: W.banded(20000, 8, seed=3), 0.0, seed=5)
    fast = _make(torch_mod, "fast", lambda: W.poisson2d(20), 1e-4, seed=6)
    ids = engine.submit([slow[2], fast[2]])
    assert engine.cancel(ids[0]) == 0
    got = engine.wait_all(ids, timeout_s=60)
    assert got[ids[0]][0].status == capi.MPCG_ECANCELED
    assert got[ids[1]][0].status == 0
    assert engine.cancel(10**12) == capi.MPCG_EINVAL
    q, act = engine.load()
    assert q == 0 and act == 0


def test_batch_many_small_systems_continuous(engine, torch_mod):
    """More systems than slots (64): requests wait for admission and join
    the running steps as earlier ones finish."""
    model = oracle.load_model(TEST_MODEL)
    rng = np.random.default_rng(12)
    fams = ["lap2d", "lap3d", "banded", "er"]
    items = []
    for i in range(96):
        fam = fams[i % 4]
        n = int(np.exp(rng.uniform(np.log(300), np.log(6000))))
        e = [1e-3, 1e-5, 0.0, -1.0][(i // 4) % 4]
        items.append((_make(torch_mod, f"{fam}{i}", lambda fam=fam, n=n, i=i: W.family_matrix(fam, n, seed=100 + i),
                            e, seed=100 + i), e))
    print(f"continuous batch of {len(items)} systems", flush=True)
    ids = []
    for k in range(0, len(items), 16):
        ids += engine.submit([it[0][2] for it in items[k:k + 16]])
        time.sleep(0.001)
    got = engine.wait_all(ids, timeout_s=300)
    for rid, ((a, b, _), e) in zip(ids, items):
        st, x = got[rid]
        if rid % 8 == 0:   # spot-check against the oracle
            _check_against_oracle(a, b, e, st, x, model)
        else:
            assert st.status == 0 and st.relres_final_true <= EPS2


def test_batch_bfs_schedule_does_not_change_results(torch_mod, monkeypatch):
    """The batched 2BFS gives the same features, and the solves the same bits,
    however its levels are scheduled: the largest frontier the one-block kernel
    takes (8 / 512 / 2,048) and the levels one of its launches may expand
    (1 / 64 / 4,096) change which kernel expands which level, how often a
    system's visited bits are rebuilt from dist and when the features arrive;
    the bands take the one-wave band sweeps or the level kernels, and the
    systems wait at their first crossing or run ahead.
    An ER graph of more than 2^20 rows takes the path that claims vertices in
    HBM (smaller systems keep their visited set in LDS); every system's
    features are checked against the oracle's 2BFS."""
    from paper_2412_08059_amd import BatchSolver
    from workloads import paper_family as PF
    gens = [("banded_30000", lambda: W.banded(30_000, 8, seed=11)),
            ("poisson2d_64", lambda: W.poisson2d(64)),
            ("er_5000", lambda: W.er_laplacian(5000, 16, seed=6)),
            ("disconnected", _disconnected),
            ("band_path_8000", lambda: PF.random_banded(8000, 3, 1.0, 1.1, seed=4)),
            ("er_1100000", lambda: W.er_laplacian(1_100_000, 16, seed=13))]
    mats = [(nm, g()) for nm, g in gens]
    print("schedules x " + ", ".join(f"{nm} (n={a.n})" for nm, a in mats), flush=True)
    schedules = [{}, {"batch_small_cap": 2048, "batch_small_levels": 4096, "batch_bfs_band": 0},
                 {"batch_small_cap": 8, "batch_small_levels": 1, "batch_group_steps": 3, "batch_bfs_rounds": 2,
                  "batch_level_grid": 96, "batch_runahead": 1, "batch_bfs_band": 0},
                 {"batch_runahead": 2}]
    runs = []
    for env in schedules:
        eng = BatchSolver(1_300_000, 40_000_000, 16, model=TEST_MODEL, tuning=env or None)
        try:
            reqs = [_make(torch_mod, nm, lambda a=a: a, 0.0, seed=30 + i)[2] for i, (nm, a) in enumerate(mats)]
            ids = eng.submit(reqs)
            got = eng.wait_all(ids, timeout_s=120)
        finally:
            eng.close()
        out = {}
        for rid, (nm, _) in zip(ids, mats):
            st, x = got[rid]
            f = st.feat
            assert st.status == 0 and st.relres_final_true <= EPS2, (env, nm, st.status)
            out[nm] = ((f.pdiam, f.bfs_t, f.bfs_u, f.n_components), st.n1, st.n2, st.eps1_class,
                       x.cpu().numpy().view(np.uint64).copy())
        print(f"  {env or 'default'}: " + ", ".join(f"{nm} pdiam={v[0][0]}" for nm, v in out.items()), flush=True)
        runs.append(out)
    for nm, a in mats:
        assert runs[0][nm][0] == oracle.pseudo_diameter(a), nm
        for r in runs[1:]:
            assert r[nm][:4] == runs[0][nm][:4], nm
            assert np.array_equal(r[nm][4], runs[0][nm][4]), nm


def _fork(M, L):
    """A tree of bandwidth 2 whose first sweep ends inside the row range: a
    path up the even rows 0 .. 2M, from 2M one branch back down the odd rows
    to row 1 and one up rows 2M + 1 .. 2M + L (M > L).  The far row of the
    sweep from row 0 is row 1, and the sweep from there splits at row 2M into
    two frontiers that move apart: wider than the band sweeps' window."""
    n = 2 * M + 1 + L
    edges = [(2 * i, 2 * i + 2) for i in range(M)] + [(2 * M, 2 * M - 1)]
    edges += [(2 * i + 1, 2 * i - 1) for i in range(M - 1, 0, -1)]
    edges += [(2 * M, 2 * M + 1)] + [(2 * M + k, 2 * M + k + 1) for k in range(1, L)]
    r = np.array([e[0] for e in edges] + [e[1] for e in edges])
    c = np.array([e[1] for e in edges] + [e[0] for e in edges])
    adj = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    lap = sp.diags(np.asarray(adj.sum(axis=1)).ravel() + 1.0) - adj
    return W.CSR.from_scipy(lap.tocsr())


def test_batch_band_2bfs_matches_oracle(torch_mod):
    """The one-wave band sweeps: features equal to the oracle's 2BFS on bands
    of half-width 1 to 31 (full and sparse), a band of 800,000 rows (its
    visited bits take 100 KB of LDS), a system of fewer rows than one word,
    and the two fallbacks -- a band that is not connected (components, then
    the level kernels) and a fork whose second sweep outgrows the window --
    each also with the band sweeps off."""
    from paper_2412_08059_amd import BatchSolver
    from workloads import paper_family as PF
    band_blocks = lambda: W.CSR.from_scipy(sp.block_diag([W.banded(3000, 4, seed=1).to_scipy(),
                                                           W.banded(2000, 6, seed=2).to_scipy()]).tocsr())
    gens = [("band_w1", lambda: PF.random_banded(20_000, 3, 1.0, 1.1, seed=5)),
            ("band_w8", lambda: W.banded(40_000, 8, seed=3)),
            ("band_w31", lambda: W.banded(9_000, 31, seed=4)),
            ("band_sparse17", lambda: PF.random_banded(30_000, 35, 0.3, 3.0, seed=6)),
            ("band_800k", lambda: W.banded(800_000, 8, seed=7)),
            ("band_tiny", lambda: W.banded(20, 3, seed=8)),
            ("band_disconnected", band_blocks),
            ("fork", lambda: _fork(3000, 2000))]
    mats = [(nm, g()) for nm, g in gens]
    for band in (1, 0):
        eng = BatchSolver(1_000_000, 30_000_000, len(mats), model=TEST_MODEL, tuning={"batch_bfs_band": band})
        try:
            reqs = [_make(torch_mod, nm, lambda a=a: a, 0.0, seed=50 + i)[2] for i, (nm, a) in enumerate(mats)]
            print(f"band sweeps {band}: " + ", ".join(f"{nm} (n={a.n})" for nm, a in mats), flush=True)
            ids = eng.submit(reqs)
            got = eng.wait_all(ids, timeout_s=300)
        finally:
            eng.close()
        for rid, (nm, a) in zip(ids, mats):
            st, _ = got[rid]
            f = st.feat
            print(f"  {nm}: status={st.status} pdiam={f.pdiam} t_feat={st.t_feat_ms:.1f} ms", flush=True)
            assert st.status == 0 and st.relres_final_true <= EPS2, (nm, st.status)
            assert (f.pdiam, f.bfs_t, f.bfs_u, f.n_components) == oracle.pseudo_diameter(a), nm


def test_batch_cancel_during_band_sweeps(torch_mod):
    """A system cancelled while its band sweeps run (a band of 2,000,000 rows:
    two sweeps of 250,000 levels) is reported cancelled -- or solved, if the
    cancel came too late -- and its slot serves the next request."""
    from paper_2412_08059_amd import BatchSolver, capi
    eng = BatchSolver(2_100_000, 40_000_000, 2, model=TEST_MODEL)
    try:
        big = _make(torch_mod, "band_2m", lambda: W.banded(2_000_000, 8, seed=9), 0.0, seed=7)
        (rid,) = eng.submit([big[2]])
        time.sleep(0.05)
        assert eng.cancel(rid) in (0, capi.MPCG_EINVAL)   # EINVAL: already reported
        st, _ = eng.wait_all([rid], timeout_s=120)[rid]
        print(f"  band_2m: status={st.status} t_feat={st.t_feat_ms:.1f} ms", flush=True)
        assert st.status in (0, capi.MPCG_ECANCELED)
        a, b, req = _make(torch_mod, "after", lambda: W.banded(5000, 8, seed=10), 0.0, seed=8)
        (rid2,) = eng.submit([req])
        st2, x2 = eng.wait_all([rid2], timeout_s=60)[rid2]
        _check_against_oracle(a, b, 0.0, st2, x2, oracle.load_model(TEST_MODEL))
    finally:
        eng.close()
