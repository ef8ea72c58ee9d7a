"""Launch parameters (tv_params) change the work decomposition only: every
setting, extremes included, gives the oracle's grids bit for bit for
single-mesh and batch calls, and so do the autotuner's runs."""
import numpy as np
import pytest

from helpers import to_numpy_words
from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu

SETTINGS = [
    {},
    {"strip_columns": 1},
    {"strip_columns": 5},
    {"strip_columns": 64},
    {"chunk_pieces": 64},
    {"chunk_pieces": 0},
    {"chunk_pieces": 65536, "strip_columns": 8},
    {"piece_cap": 1},
    {"piece_cap": 3},
    {"tile_cols_log2": 3},
    {"tile_cols_log2": 4, "min_tiles": 1},
    {"min_tiles": 1 << 20},
    {"wgs_per_cu": 1},
    {"wgs_per_cu": 8},
    {"cull_columns": 0},
    {"cull_columns": 1024},
    {"tile_cols_log2": 3, "chunk_pieces": 64, "strip_columns": 3, "piece_cap": 1, "wgs_per_cu": 1},
]


def banner(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def cases(oracle_mod):
    import torch

    ms = [synth.workload_small(),
          synth.make_mesh(6, 0.3, 128, "ellipsoids", 2, 9101),  # tets spanning many tiles
          synth.make_mesh(24, 0.35, 256, "ellipsoids", 3, 9102)]
    ms += synth.workload_batch(first=6, workers=1)
    items = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tets).cuda(), m.dims, m.bbox, False)
             for m in ms]
    want = [oracle_mod.voxelize_mesh(m) for m in ms]
    return ms, items, want


@pytest.mark.parametrize("setting", SETTINGS, ids=[",".join(f"{k}={v}" for k, v in s.items()) or "defaults"
                                                   for s in SETTINGS])
def test_setting_matches_oracle(cases, setting):
    import paper_2106_01326_amd as tv

    ms, items, want = cases
    banner(f"params {setting}")
    try:
        tv.set_params("single", **setting)
        for i, (v, t, dims, bbox, q) in enumerate(items[:3]):
            grid, ws = tv.voxelize(v, t, dims, bbox)
            assert np.array_equal(to_numpy_words(grid), want[i]), f"single mesh {i}"
            assert tv.fetch_status(ws) == tv.TV_OK
        tv.set_params("batch", **setting)
        b = tv.Batch(items)
        for g in b.grids:
            g.fill_(-1)
        for i, g in enumerate(b.run()):
            assert np.array_equal(to_numpy_words(g), want[i]), f"batch mesh {i}"
        # a prepared batch keeps the parameters of its prepare call
        b.prepare()
        tv.set_params("batch", None)
        for g in b.grids:
            g.fill_(-1)
        for i, g in enumerate(b.run_prepared()):
            assert np.array_equal(to_numpy_words(g), want[i]), f"prepared batch mesh {i}"
    finally:
        tv.set_params("single", None)
        tv.set_params("batch", None)


def test_autotuner_runs_and_caches(cases, tmp_path):
    import paper_2106_01326_amd as tv
    from paper_2106_01326_amd import tune

    ms, items, want = cases
    cache = str(tmp_path / "tune.json")
    v, t, dims, bbox, _ = items[2]
    banner("tune_single on a 256^3 mesh")
    tv.set_params("single", strip_columns=5)  # a setting of the caller's, restored after the search
    r = tune.tune_single(v, t, dims, bbox, reps=1, cache=cache)
    assert tv.get_params("single") == dict(tv.default_params("single"), strip_columns=5)
    tv.set_params("single", None)
    assert r["ms_best"] <= r["ms_default"]
    for f, val in r["params"].items():
        assert val == tv.default_params("single")[f] or val in tune.CANDIDATES[f]
    assert len(r["log"]) > 10
    assert tune.apply_cached("single", r["key"], cache)
    try:
        grid, _ = tv.voxelize(v, t, dims, bbox)
        assert np.array_equal(to_numpy_words(grid), want[2])
    finally:
        tv.set_params("single", None)
    banner("tune_batch on nine meshes")
    b = tv.Batch(items)
    rb = tune.tune_batch(b, reps=1, cache=cache)
    assert rb["ms_best"] <= rb["ms_default"]
    assert tune.cached(rb["key"], cache)["params"] == rb["params"]
    assert tv.get_params("batch") == tv.default_params("batch")


def test_batch_with_many_tiles(oracle_mod):
    """Many tiles in one call (the queue-layout scan runs 19 rounds of 1024
    tiles): 300 meshes on 64^3 grids cut into 8x8-column tiles."""
    import torch

    import paper_2106_01326_amd as tv

    ms = [synth.make_mesh(4 + (i % 5), 0.3, 64, "ellipsoids", 1 + i % 3, 9300 + i) for i in range(300)]
    banner(f"batch of {len(ms)} meshes with 8x8-column tiles")
    try:
        tv.set_params("batch", tile_cols_log2=3, min_tiles=1 << 20)
        items = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tets).cuda(), m.dims, m.bbox, False)
                 for m in ms]
        b = tv.Batch(items)
        plan = b.prepare()
        assert plan.ntiles > 16384
        for i, g in enumerate(b.run_prepared()):
            assert np.array_equal(to_numpy_words(g), oracle_mod.voxelize_mesh(ms[i])), f"mesh {i}"
            assert b.status(i) == tv.TV_OK
    finally:
        tv.set_params("batch", None)
