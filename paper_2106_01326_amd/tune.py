"""Autotuner of the tile pipeline's launch parameters (tv_params).

The parameters only decompose the work (tile edge, tiles per lone grid,
pieces per queue task, columns per lane task, the large-tet threshold and the
persistent workgroup count); every setting gives the same grid bit for bit.
The tuner measures candidates on the device and keeps the fastest:

* one coordinate at a time, starting from the library defaults, each
  candidate timed with HIP events on the launch stream (median of `reps`
  calls after one warm-up call);
* every candidate's grids are compared word for word with the grids of the
  default setting, and a difference raises (it would be a library bug);
* results go to a JSON cache keyed by GPU architecture, call kind and size
  class, so a later process can apply them with `apply_cached`.

Calls of the library run through the C ABI; this module only chooses the
values handed to tv_set_params.
"""
from __future__ import annotations

import json
import math
import os

import paper_2106_01326_amd as tv

# values tried per field (the default is always among them)
CANDIDATES = {
    "strip_columns": (4, 6, 8, 12, 16),
    "chunk_pieces": (0, 256, 512, 1024, 2048, 4096, 8192, 16384),
    "tile_cols_log2": (5, 4),
    "min_tiles": (256, 512, 1024, 2048),
    "piece_cap": (2, 4, 8),
    "wgs_per_cu": (1, 2, 3),
    "cull_columns": (1, 3, 6, 12),
}
# fields not tuned for batch calls (each mesh keeps the largest tiles)
BATCH_SKIP = ("min_tiles",)


def default_cache_path() -> str:
    return os.environ.get("TV_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tetvox",
                                                        "tune.json"))


def _arch(torch) -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def size_class_single(nt: int, dims) -> str:
    return f"nt2^{max(0, round(math.log2(max(nt, 1))))}:dims{dims[0]}x{dims[1]}x{dims[2]}"


def size_class_batch(meshes: int, nt: int) -> str:
    return f"n2^{max(0, round(math.log2(max(meshes, 1))))}:nt2^{max(0, round(math.log2(max(nt, 1))))}"


def _time(torch, fn, reps: int) -> float:
    """Median milliseconds of `fn` over `reps` calls (after one warm-up)."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def _search(torch, which: str, run, reps: int, fields, rounds: int = 1):
    """Coordinate search over `fields`.  `run()` makes one call with the
    parameters in force (reallocating its workspace when needed) and returns
    its grids.  Returns (best params, ms of the defaults, ms of the best, log);
    the parameters in force before the search are restored afterwards."""
    before = tv.get_params(which)
    tv.set_params(which, None)
    base = tv.get_params(which)
    ref = [g.clone() for g in run()]
    torch.cuda.synchronize()
    ms_default = _time(torch, run, reps)
    best, best_ms = dict(base), ms_default
    log = [{"params": dict(base), "ms": ms_default}]
    try:
        for _ in range(rounds):
            for field in fields:
                for value in CANDIDATES[field]:
                    if value == best[field]:
                        continue
                    trial = dict(best)
                    trial[field] = value
                    tv.set_params(which, trial)
                    out = run()
                    torch.cuda.synchronize()
                    for i, (a, b) in enumerate(zip(out, ref)):
                        if not torch.equal(a, b):
                            raise RuntimeError(f"parameters {trial} changed grid {i}")
                    ms = _time(torch, run, reps)
                    log.append({"params": trial, "ms": ms})
                    if ms < best_ms:
                        best, best_ms = trial, ms
    finally:
        tv.set_params(which, before)
    return best, ms_default, best_ms, log


def _store(cache, key, entry):
    path = cache or default_cache_path()
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_single(verts, tets, dims, bbox=None, qverts=False, reps=5, rounds=1, cache=None, store=True):
    """Tunes the single-mesh parameters on one mesh (device tensors).
    Returns {"key", "params", "ms_default", "ms_best", "log"}; the result is
    written to the cache unless store is False.  The parameters in force
    before the call are restored afterwards."""
    torch = tv._torch()
    nv, nt = int(verts.shape[0]), int(tets.shape[0])
    grid = tv.alloc_grid(dims, verts.device)
    state = {"ws": None}

    def run():
        need = tv.workspace_bytes(nv, nt, dims)
        if state["ws"] is None or state["ws"].numel() < need:
            state["ws"] = tv.alloc_workspace(need, verts.device)
        tv.voxelize(verts, tets, dims, bbox, qverts=qverts, grid=grid, workspace=state["ws"])
        return [grid]

    best, ms0, ms1, log = _search(torch, "single", run, reps, list(CANDIDATES), rounds)
    key = f"{_arch(torch)}:single:{size_class_single(nt, dims)}"
    entry = {"key": key, "params": best, "ms_default": ms0, "ms_best": ms1, "log": log}
    if store:
        _store(cache, key, {"params": best, "ms_default": ms0, "ms_best": ms1})
    return entry


def tune_batch(batch, reps=3, rounds=1, cache=None, store=True):
    """Tunes the batch parameters on a tv.Batch (its grids are overwritten).
    Returns as tune_single."""
    torch = tv._torch()

    def run():
        batch.resize_workspace()
        return batch.run()

    fields = [f for f in CANDIDATES if f not in BATCH_SKIP]
    best, ms0, ms1, log = _search(torch, "batch", run, reps, fields, rounds)
    nt = sum(int(it[1].shape[0]) for it in batch.items)
    key = f"{_arch(torch)}:batch:{size_class_batch(batch.n, nt)}"
    entry = {"key": key, "params": best, "ms_default": ms0, "ms_best": ms1, "log": log}
    if store:
        _store(cache, key, {"params": best, "ms_default": ms0, "ms_best": ms1})
    return entry


def cached(key, cache=None):
    """The cached entry for `key`, or None."""
    path = cache or default_cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(key)


def apply_cached(which, key, cache=None) -> bool:
    """Sets the parameters cached under `key` (True), or leaves them (False)."""
    e = cached(key, cache)
    if e is None:
        return False
    tv.set_params(which, e["params"])
    return True
