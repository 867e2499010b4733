"""The autotuner's parameters through the C ABI: every candidate leaves the
results unchanged bit for bit (solves and features), and a loaded table is
applied by the nearest-class rule.  The packaged table must load."""

import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TEST_MODEL = os.path.join(GOLDEN, "knn_model_test.txt")


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def dev(a):
    from paper_2412_08059_amd import DeviceCSR
    return DeviceCSR.from_host(a)


CASES = {
    "varcoef3d_20": lambda: W.varcoef3d(20, seed=3),
    "banded_30k": lambda: W.banded(30_000, 8, seed=3),
    "er_100k_wide": lambda: W.er_laplacian(100_000, 16, seed=4),   # 32-bit columns: the split is a candidate
}


@pytest.mark.parametrize("name", list(CASES))
def test_every_sell_candidate_gives_the_same_bits(torch_mod, name):
    from paper_2412_08059_amd import Solver
    from paper_2412_08059_amd import autotune as at
    a = CASES[name]()
    _, b = W.rhs(a, seed=5)
    A, B = dev(a), torch_mod.from_numpy(b).cuda()
    s = Solver(a.n, a.nnz, model=TEST_MODEL, tuning=None)
    ref = None
    idx16 = 1 if at.band_of(a) < 32768 else 0
    try:
        for cand in at.sell_candidates(idx16):
            for stream in (0, 1):   # cached or nontemporal matrix loads
                s.set_tuning(dict(zip(("sell_batch", "sell_whole_batch", "sell_split"), cand), sell_stream=stream))
                out = []
                for e1 in (1e-5, 0.0):
                    st, x, S = s.solve(A, B, e1, 1e-10)
                    assert st == 0
                    out.append((S.n1, S.n2, S.eps1_class, x.cpu().numpy().view(np.uint64).copy()))
                print(f"{name} {cand} stream {stream}: n1/n2 {[o[:2] for o in out]}", flush=True)
                if ref is None:
                    ref = out
                for o, r in zip(out, ref):
                    assert o[:3] == r[:3] and np.array_equal(o[3], r[3]), (cand, stream)
    finally:
        s.close()


@pytest.mark.parametrize("name", ["varcoef3d_20", "banded_30k"])
def test_every_bfs_candidate_gives_the_same_features(torch_mod, name):
    from paper_2412_08059_amd import Solver
    a = CASES[name]()
    _, b = W.rhs(a, seed=5)
    A, B = dev(a), torch_mod.from_numpy(b).cuda()
    s = Solver(a.n, a.nnz, tuning=None)
    got = set()
    try:
        for grid in (1, 64, 256):
            for persist in (0, 1):
                for dia, tiles in ((0, 0), (2, 0), (2, 1)):   # queue kernels, diagonal levels, tiles
                    s.set_tuning(dict(bfs_grid=grid, bfs_grid_shared=grid, bfs_persist=persist, bfs_dia=dia,
                                      bfs_dia_tiles=tiles))
                    st, f = s.features(A, B, 20)
                    assert st == 0
                    got.add((f.pdiam, f.bfs_t, f.bfs_u, f.n_components, f.k0_used, f.v))
    finally:
        s.close()
    assert len(got) == 1, got


def test_table_lookup_and_overrides(torch_mod, tmp_path):
    import torch
    from paper_2412_08059_amd import Solver, capi
    from paper_2412_08059_amd import autotune as at
    props = torch.cuda.get_device_properties(0)
    arch, cu = props.gcnArchName.split(":")[0], props.multi_processor_count
    mk = lambda bt, w, sp, g, dia=1: dict(sell_batch=bt, sell_whole_batch=w, sell_split=sp, bfs_grid=g,
                                           bfs_grid_shared=32, bfs_persist=0, bfs_dia=dia, bfs_dia_tiles=1,
                                           sell_stream=-1)
    rows = {(arch, cu, 1, 3, 12): mk(8, 0, -1, 64), (arch, cu, 1, 3, 20): mk(4, 3, -1, 256, dia=0),
            (arch, cu, 0, 4, 20): mk(8, 2, 1, 128), ("gfx000", cu, 1, 3, 16): mk(8, 3, 0, 1)}
    batch = (arch, cu, dict(batch_group_steps=3, batch_bfs_rounds=5, batch_small_cap=100, batch_small_levels=7,
                            batch_level_grid=99))
    path = tmp_path / "t.txt"
    path.write_text(at.format_table(rows, batch))
    s = Solver(100, 1000, tuning=str(path))
    try:
        # 7-point stencil class (16-bit, lenlog 3): nearest log2(n) wins, ties to the smaller
        assert s.tuning_for(2 ** 13, 7 * 2 ** 13, 64)["sell_batch"] == 8          # nlog 13 -> entry 12
        assert s.tuning_for(2 ** 16, 7 * 2 ** 16, 64)["bfs_grid"] == 64            # nlog 16: 12 and 20 tie -> 12
        assert s.tuning_for(2 ** 21, 7 * 2 ** 21, 64)["sell_whole_batch"] == 3     # nlog 21 -> entry 20
        assert s.tuning_for(2 ** 21, 7 * 2 ** 21, 64)["bfs_dia"] == 0
        assert s.tuning_for(2 ** 20, 16 * 2 ** 20, 40000)["sell_split"] == 1       # 32-bit, lenlog 4
        # no entry for this class (lenlog 1): the defaults
        d = s.tuning_for(1000, 2000, 1)
        assert (d["sell_batch"], d["sell_whole_batch"], d["sell_split"], d["bfs_grid"]) == (4, 1, -1, 128)
        assert (d["bfs_dia"], d["bfs_dia_tiles"], d["sell_stream"]) == (1, 1, -1)
        assert (d["batch_runahead"], d["batch_bfs_band"]) == (0, 1)
        # a malformed table is refused and the loaded one stays
        bad = tmp_path / "bad.txt"
        bad.write_text("mpcg-tune 1\nsolve gfx950 256 1 3\n")
        assert capi.mpcg_load_tuning(s.ctx, str(bad)) == capi.MPCG_EINVAL
        bad.write_text("mpcg-tune 1\nbatch gfx950 256 8 4 512 64 1024 3 1\n")   # runahead out of range
        assert capi.mpcg_load_tuning(s.ctx, str(bad)) == capi.MPCG_EINVAL
        assert s.tuning_for(2 ** 13, 7 * 2 ** 13, 64)["sell_batch"] == 8
        # explicit values win over the table; None goes back to it
        s.set_tuning({"sell_batch": 4, "bfs_grid": 17})
        assert s.tuning_for(2 ** 13, 7 * 2 ** 13, 64)["bfs_grid"] == 17
        assert capi.mpcg_set_tuning(s.ctx, {"sell_batch": 5}) == capi.MPCG_EINVAL
        assert capi.mpcg_set_tuning(s.ctx, {"bfs_dia": 3}) == capi.MPCG_EINVAL
        assert capi.mpcg_set_tuning(s.ctx, {"bfs_dia_tiles": 2}) == capi.MPCG_EINVAL
        assert capi.mpcg_set_tuning(s.ctx, {"sell_stream": 2}) == capi.MPCG_EINVAL
        assert capi.mpcg_set_tuning(s.ctx, {"batch_runahead": 3}) == capi.MPCG_EINVAL
        assert capi.mpcg_set_tuning(s.ctx, {"batch_bfs_band": -1}) == capi.MPCG_EINVAL
    finally:
        s.close()
    # the options' explicit product variant overrides the table's split
    s2 = Solver(100, 1000, tuning=str(path), spmv_variant=1)
    try:
        assert s2.tuning_for(2 ** 20, 16 * 2 ** 20, 40000)["sell_split"] == 0
    finally:
        s2.close()


def test_packaged_table_loads(torch_mod):
    from paper_2412_08059_amd import DEFAULT_TUNING, Solver, capi
    if not os.path.exists(DEFAULT_TUNING):
        pytest.skip("no packaged tuning table")
    s = Solver(100, 1000, tuning=None)
    try:
        assert capi.mpcg_load_tuning(s.ctx, DEFAULT_TUNING) == capi.MPCG_OK
    finally:
        s.close()
