"""Host-side parts of the autotuner: the class key (the same bucketing as the
library's tune.cpp), candidate lists, selection and the table text."""

import numpy as np
import pytest

import workloads as W

at = pytest.importorskip("paper_2412_08059_amd.autotune")


def test_class_key_buckets():
    assert at.nlog(1) == 0 and at.nlog(2) == 1 and at.nlog(4095) == 11 and at.nlog(4096) == 12
    assert at.nlog(2_097_152) == 21
    # mean row length: 7-point stencil ~6.95 -> log2 2.8 -> 3; 17-entry band -> 4.09 -> 4
    assert at.lenlog(2_097_152, 14_581_760) == 3 and at.lenlog(1_000_000, 16_999_928) == 4
    # halves go up (C's lround): mean 2^2.5 = 5.657
    assert at.lenlog(1000, int(np.ceil(1000 * 2 ** 2.5))) == 3
    assert at.lenlog(10, 0) == 0
    band = W.banded(5000, 8, seed=0)
    er = W.er_laplacian(100_000, 16, seed=0)
    assert at.band_of(band) == 8 and at.band_of(er) >= 32768
    assert at.class_key("gfx950", 256, band)[2:] == (1, 4, 12)
    assert at.class_key("gfx950", 256, er)[2] == 0


def test_candidates_and_choice():
    c16, c32 = at.sell_candidates(1), at.sell_candidates(0)
    assert len(c16) == 8 and all(sp == -1 for _, _, sp in c16)
    assert len(c32) == 16 and {sp for _, _, sp in c32} == {0, 1}
    assert at.choose_min({"a": 3.0, "b": 1.0, "c": 1.0}) == "b"


def test_table_roundtrip():
    rows = {("gfx950", 256, 1, 3, 21): dict(sell_batch=4, sell_whole_batch=1, sell_split=-1, bfs_grid=128,
                                            bfs_grid_shared=64, bfs_persist=0, bfs_dia=1, bfs_dia_tiles=1,
                                            sell_stream=-1),
            ("gfx950", 256, 0, 4, 20): dict(sell_batch=8, sell_whole_batch=3, sell_split=1, bfs_grid=256,
                                            bfs_grid_shared=32, bfs_persist=1, bfs_dia=2, bfs_dia_tiles=0,
                                            sell_stream=1)}
    batch = ("gfx950", 256, dict(batch_group_steps=4, batch_bfs_rounds=4, batch_small_cap=256,
                                 batch_small_levels=64, batch_level_grid=512, batch_runahead=1,
                                 batch_bfs_band=0))
    text = at.format_table(rows, batch, comment="test")
    assert text.startswith("mpcg-tune 1\n")
    r2, b2 = at.parse_table(text)
    assert r2 == rows and b2 == batch
    # rows written before the last three fields take their defaults (1, 1, -1)
    old_row = "mpcg-tune 1\nsolve gfx950 256 1 3 21 4 1 -1 128 64 0\n"
    r3, _ = at.parse_table(old_row)
    # a batch row written before the last two fields takes their defaults (hold, band 2BFS on)
    _, b4 = at.parse_table("mpcg-tune 1\nbatch gfx950 256 8 4 512 64 1024\n")
    assert b4[2]["batch_runahead"] == 0 and b4[2]["batch_bfs_band"] == 1
    assert r3[("gfx950", 256, 1, 3, 21)]["bfs_dia"] == 1 and r3[("gfx950", 256, 1, 3, 21)]["bfs_dia_tiles"] == 1
    assert r3[("gfx950", 256, 1, 3, 21)]["sell_stream"] == -1
    with pytest.raises(ValueError):
        at.parse_table("mpcg-tune 2\n")
