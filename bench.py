#!/usr/bin/env python3
"""Benchmark of the voxelization hot path on one MI355X.

A step is one complete voxelization of one mesh (grid clear, vertex snap,
per-tet setup and column-span voxelization) with the inputs already resident
in HBM.  Prints ONE JSON line:

  metric/value/unit   tets voxelized per second (whole job), plus meshes/s
  roofline            dominant kernel (voxelize) vs the VALU peak
  cpu_baseline        the CPU oracle timed on a bounded sample of the same
                      workload on the host's cores (rank 0, N=1 only)

Workloads (seeded synthetic Kuhn meshes, see paper_2106_01326_amd/synth.py):
  large   128^3 cubes x 6 tets, jitter 0.45, 6 ellipsoids, 1024^3 grid, fp32 (default)
  medium  64^3 cubes x 6 tets, jitter 0.3, 3 ellipsoids, 256^3 grid, int32 lattice verts
  small   8^3 cubes x 6 tets, jitter 0.2, sphere, 32^3 grid, fp32
  batch   1024 meshes of uneven size (cubes per axis U{4..48}, jitter U[0,0.4],
          1-4 ellipsoids, 32^3 or 64^3 grids): one batched call vs the
          per-mesh loop, meshes/s and tets/s
  serving Poisson stream of requests (90% batch-distribution meshes, 10%
          medium-shape meshes at 256^3) through the continuous-batching
          server at 0.5/0.7/0.9 x its measured capacity: p50/p99 latency and
          meshes/s
  tune    the autotuner (paper_2106_01326_amd/tune.py) on the large, medium
          and batch workloads: default vs tuned milliseconds and parameters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LAT = 1 << 16
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes/clk x 2.4 GHz = 39.3 T lane-ops/s
# Algorithmic VALU lane-operations of the exact column-span formulation:
SETUP_OPS_PER_TET = 170  # box (min/max/shift/clamp) + 4 faces (edges, cross, orient, tie, base, scales, 1/sz)
OPS_PER_COLUMN = 24      # 4 faces x (evaluate, quotient estimate, round, exact check, merge) + run write


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Synthetic inputs are generated once per process and before the process
# touches the GPU (see pregenerate); the worker pools that build many meshes
# start fresh processes.
_MESHES = {}


def _memo(key, fn):
    if key not in _MESHES:
        t0 = time.perf_counter()
        _MESHES[key] = fn()
        log(f"generated {key} in {time.perf_counter() - t0:.1f} s")
    return _MESHES[key]


CACHE_DIR = None  # --cache-dir: single-mesh workloads saved as .npz and reused


def _cached(name, gen):
    """The mesh from the cache directory when it holds it, else generated
    (and saved there).  The file name carries the workload and the seed's
    default, and the arrays are compared with nothing: delete the directory
    after changing the generator."""
    from paper_2106_01326_amd import synth

    if not CACHE_DIR:
        return gen()
    path = os.path.join(CACHE_DIR, f"{name}.npz")
    if os.path.exists(path):
        d = np.load(path, allow_pickle=False)
        m = synth.Mesh(tets=d["tets"], dims=tuple(int(x) for x in d["dims"]), bbox=(d["lo"], d["hi"]),
                       meta=json.loads(str(d["meta"])))
        if "verts" in d.files:
            m.verts = d["verts"]
        else:
            m.qverts = d["qverts"]
        return m
    m = gen()
    os.makedirs(CACHE_DIR, exist_ok=True)
    arrs = {"tets": m.tets, "dims": np.array(m.dims), "lo": m.bbox[0], "hi": m.bbox[1],
            "meta": np.array(json.dumps(m.meta))}
    arrs["verts" if m.verts is not None else "qverts"] = m.verts if m.verts is not None else m.qverts
    np.savez(path + ".tmp.npz", **arrs)
    os.replace(path + ".tmp.npz", path)
    return m


def make_workload(name):
    from paper_2106_01326_amd import synth

    gen = {"large": synth.workload_large, "medium": synth.workload_medium, "small": synth.workload_small}
    if name not in gen:
        raise SystemExit(f"unknown workload {name}")
    return _memo(name, lambda: _cached(name, gen[name]))


def batch_meshes(count):
    from paper_2106_01326_amd import synth

    return _memo(f"batch{count}", lambda: synth.workload_batch(count=count, workers=gen_workers()))


def serving_pool():
    """512 batch-distribution meshes (seed 4) and 32 medium-shape fp32
    meshes (seeds drawn from the same stream as the arrivals)."""
    from paper_2106_01326_amd import synth

    def make():
        rng = np.random.default_rng(4)
        small = synth.workload_batch(count=512, seed=4, workers=gen_workers())
        seeds = [int(x) for x in rng.integers(0, 2**31, size=32)]
        big = synth.pool_map(synth.medium_shape_fp32, seeds, gen_workers())
        return small + big

    return _memo("serving_pool", make)


def gen_workers():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    w = int(os.environ.get("TV_BENCH_GEN_WORKERS", "0")) or min(16, n)
    return max(1, w)


def host_cores():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pregenerate(args):
    """Builds every synthetic input the chosen workload uses, before the
    first GPU call."""
    w = args.workload
    if w in ("large", "medium", "small"):
        make_workload(w)
        if w == "large" and not args.no_extras:
            batch_meshes(args.batch_meshes)
            if args.with_serving:
                serving_pool()
    elif w == "batch":
        batch_meshes(args.batch_meshes)
    elif w == "serving":
        serving_pool()
    elif w in ("grids", "quality", "bricks"):
        make_workload("large")
        if w == "quality":
            make_workload("medium")
    elif w == "tune":
        make_workload("large")
        make_workload("medium")
        batch_meshes(args.batch_meshes)


def workload_config(name, m):
    return {"workload": {"large": "large single mesh, 1024^3 grid", "medium": "medium single mesh, 256^3 grid",
                         "small": "small single mesh, 32^3 grid"}[name],
            "cubes_per_axis": m.meta["n"], "jitter": m.meta["delta"], "keep": m.meta["keep"],
            "ellipsoids": m.meta["k"], "grid": list(m.dims), "vert_format": m.fmt,
            "tets": m.nt, "verts": m.nv, "tets_before_keep": m.meta["tets_before_keep"], "seed_index": True}


def candidate_work(q, tets, dims):
    """(#tets with a non-empty candidate box, #candidate columns, #candidate
    centers) from the lattice vertices -- counts only, for the roofline."""
    p = q[tets]  # [nt,4,3]
    mn = p.min(axis=1).astype(np.int64)
    mx = p.max(axis=1).astype(np.int64)
    half = np.array([(LAT // 2) // d for d in dims], dtype=np.int64)
    lo = np.maximum(0, -((half - mn) // (2 * half)))
    hi = np.minimum(np.array(dims) - 1, (mx - half) // (2 * half))
    ext = np.maximum(hi - lo + 1, 0)
    nonempty = np.all(ext > 0, axis=1)
    cols = (ext[:, 0] * ext[:, 1])[nonempty]
    cand = (ext[:, 0] * ext[:, 1] * ext[:, 2])[nonempty]
    return int(nonempty.sum()), int(cols.sum()), int(cand.sum())


# the sources that build and launch the tile kernel (its counters go stale
# when one of these changes)
TILE_KERNEL_SOURCES = ("tv_kernels.hip", "tv_kernels.h", "tv_common.h", "tv_workspace.h", "tv_api.hip")


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_01326_amd", "csrc")
    for fn in TILE_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per voxelize launch from the committed counter summary, or
    None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_voxelize_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def valu_counters_from_profiles(workload, kept_columns=None):
    """VALU counters of the tile kernel from the committed rocprofv3 --pmc
    summary, or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"valu_voxelize_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec.get("summary")


def cpu_baseline(m, gpu_words_fn, target_s=12.0):
    """The oracle, as it stands, on a bounded sample (the first tets of the
    mesh), on all host cores; the GPU path runs the same sample and the two
    grids are compared bit for bit."""
    import oracle

    cores = host_cores()
    q = oracle.snap(m.verts, *m.bbox) if m.verts is not None else m.qverts
    # grow the sample until one run takes about target_s: a short probe
    # underestimates the rate (grid clearing and thread start-up dominate it)
    n = min(m.nt, 20000)
    while True:
        sample = m.tets[:n]
        t0 = time.perf_counter()
        if m.verts is not None:
            want = oracle.voxelize_q(oracle.snap(m.verts, *m.bbox), sample, m.dims, threads=cores)
        else:
            want = oracle.voxelize_q(q, sample, m.dims, threads=cores)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or n == m.nt:
            break
        n = int(min(m.nt, n * min(16.0, max(2.0, 0.9 * target_s / max(dt, 1e-6)))))
    got = gpu_words_fn(sample)
    exact = bool(np.array_equal(got, want))
    # one thread, on a sample sized for about a third of target_s
    n1 = max(1000, min(m.nt, int(n / dt * target_s / 3 / cores)))
    t0 = time.perf_counter()
    oracle.voxelize_q(q if m.verts is None else oracle.snap(m.verts, *m.bbox), m.tets[:n1], m.dims, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "tets/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {m.nt} tets (snap + voxelize, {dt:.1f} s wall)",
            "seconds": dt, "gpu_bit_exact_on_sample": exact,
            "value_1thread": n1 / dt1, "sample_1thread": f"first {n1} tets on one thread ({dt1:.1f} s wall)",
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}


def tile_roofline(torch, tv, items, meshes, vox_ms):
    """The tile kernel against the VALU peak for a call over `meshes`
    (device vertex tensors in items[i][0]): algorithmic ops from the lattice
    vertices (snapped on the device), divided by the measured voxelize-stage
    time per call."""
    ne = cols = 0
    for (v, _, dims, bbox, _), m in zip(items, meshes):
        q = tv.snap(v, bbox).cpu().numpy()
        a, b, _ = candidate_work(q, m.tets, dims)
        ne += a
        cols += b
    ops = SETUP_OPS_PER_TET * ne + OPS_PER_COLUMN * cols
    achieved = ops / (vox_ms * 1e-3) / 1e12 if vox_ms > 0 else None
    return {"bound": "alu", "kernel": "k_tile_voxelize", "achieved": achieved, "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS if achieved else None, "traffic": None,
            "kernel_ms": vox_ms, "ops_per_launch": ops,
            "units": {"tets_nonempty": ne, "candidate_columns": cols}}


def batch_core(args, torch, tv, meshes, steps, warmup, cpu=True):
    """Batched voxelization of the uneven batch vs a loop of single-mesh
    calls (the per-mesh baseline: back to back on one stream, one final
    sync -- its best case); returns the measurements as a dict."""
    nt = sum(m.nt for m in meshes)
    dev = torch.device("cuda:0")
    items = [(torch.from_numpy(m.verts).to(dev), torch.from_numpy(m.tets).to(dev), m.dims, m.bbox, False)
             for m in meshes]
    stream = torch.cuda.current_stream()
    batch = tv.Batch(items)
    for _ in range(warmup):
        batch.run(stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        batch.run(stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1) / steps
    # stage times from a separate profiled pass
    tv.profile_read()
    tv.profile_enable(True)
    for _ in range(max(2, min(steps, 5))):
        batch.run(stream=stream)
    torch.cuda.synchronize()
    tv.profile_enable(False)
    stages, calls = tv.profile_read()
    bad = [i for i in range(len(meshes)) if batch.status(i) != tv.TV_OK]
    assert not bad, f"status errors in meshes {bad[:5]}"
    log(f"batched: {ms_batch:.3f} ms per batch; profiled stages (ms per call) "
        f"{ {k: round(v_ / max(calls, 1), 4) for k, v_ in stages.items()} }")

    # the same batch prepared once and replayed as a captured HIP graph
    # (tv_batch_prepare, then tv_batch_run inside torch's graph capture)
    ref = [g.clone() for g in batch.grids]
    batch.prepare()
    batch.run_prepared()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run_prepared()
    graph.replay()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_graph = ev0.elapsed_time(ev1) / steps
    graph_same = all(torch.equal(a, b) for a, b in zip(ref, batch.grids))
    del graph, ref
    log(f"graph replay of the prepared batch: {ms_graph:.3f} ms per batch; identical={graph_same}")

    # per-mesh loop with preallocated grids and workspaces
    grids = [tv.alloc_grid(m.dims, dev) for m in meshes]
    wss = [tv.alloc_workspace(tv.workspace_bytes(m.nv, m.nt, m.dims), dev) for m in meshes]

    def loop():
        for (v, t, dims, bbox, _), g, w in zip(items, grids, wss):
            tv.voxelize(v, t, dims, bbox, grid=g, workspace=w, stream=stream)

    loop()
    torch.cuda.synchronize()
    reps = max(1, min(3, steps))
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(reps):
        loop()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_loop = ev0.elapsed_time(ev1) / reps
    wall_loop = (time.perf_counter() - t0) * 1e3 / reps
    same = all(torch.equal(a, b) for a, b in zip(grids, batch.grids))
    log(f"per-mesh loop: {ms_loop:.3f} ms per pass (host wall {wall_loop:.3f} ms); identical={same}")
    res = {"meshes": len(meshes), "tets": nt, "ms_per_batch": ms_batch,
           "meshes_per_s": len(meshes) / (ms_batch * 1e-3), "tets_per_s": nt / (ms_batch * 1e-3),
           "per_mesh_loop": {"meshes_per_s": len(meshes) / (ms_loop * 1e-3), "ms_per_pass": ms_loop,
                             "host_wall_ms_per_pass": wall_loop},
           "batched_over_per_mesh": ms_loop / ms_batch, "bit_identical_to_per_mesh": bool(same),
           "graph_replay": {"ms_per_batch": ms_graph, "meshes_per_s": len(meshes) / (ms_graph * 1e-3),
                            "bit_identical": bool(graph_same)},
           "stage_ms": {k: v_ / max(calls, 1) for k, v_ in stages.items()}}
    res["roofline"] = tile_roofline(torch, tv, items, meshes, stages.get("voxelize", 0.0) / max(calls, 1))
    # the batch's grids exported to one CNN input tensor per resolution
    exp = tv.Export([(g, m.dims) for g, m in zip(batch.grids, meshes)])
    res["export"] = {}
    for r_ in (32, 64):
        out_t = torch.empty((len(meshes), r_, r_, r_), dtype=torch.float32, device=dev)
        ws_e = tv.alloc_workspace(int(tv.load_library().tv_export_workspace_bytes(len(meshes))), dev)
        exp.run(r_, "fraction", out=out_t, workspace=ws_e, stream=stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            exp.run(r_, "fraction", out=out_t, workspace=ws_e, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_e = ev0.elapsed_time(ev1) / steps
        in_bytes = sum(tv.grid_words(m.dims) * 4 for m in meshes)
        res["export"][f"res{r_}_f32"] = {"ms": ms_e, "out_bytes": out_t.numel() * 4,
                                         "GB_per_s": (in_bytes + out_t.numel() * 4) / (ms_e * 1e-3) / 1e9}
        del out_t, ws_e
    del exp
    log(f"export: {res['export']}")
    if cpu:
        res["cpu_baseline"] = cpu_baseline_batch(meshes, batch, args.cpu_seconds)
    del grids, wss, items, batch
    return res


def bench_batch(args, torch, tv):
    """The uneven batch workload as its own line (meshes/s batched)."""
    meshes = batch_meshes(args.batch_meshes)
    r = batch_core(args, torch, tv, meshes, args.steps, args.warmup, cpu=not args.no_cpu_baseline)
    out = {"metric": "meshes/s (batched)", "value": r["meshes_per_s"], "unit": "meshes/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_batch"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes)",
           "config": {"workload": "uneven batch of small meshes", "meshes": len(meshes), "tets": r["tets"],
                      "grids": "32^3 or 64^3", "vert_format": "f32"}}
    for k in ("tets_per_s", "per_mesh_loop", "batched_over_per_mesh", "bit_identical_to_per_mesh",
              "graph_replay", "stage_ms", "roofline", "export"):
        out[k] = r[k]
    out["cpu_baseline"] = r.get("cpu_baseline")
    print(json.dumps(out), flush=True)


def serving_core(args, torch, tv, pool_meshes, runs=3):
    """Poisson arrivals through the server.  Inputs are pre-staged in pinned
    host memory (as a serving front end receiving into pinned buffers
    would); grids stay on the device until the client releases them.

    Sustained capacity is the highest offered Poisson rate, on a grid of
    rates, that the server keeps up with (achieved >= 97% of offered over
    the run); p50/p99 are then measured at 0.5/0.7/0.9 x that rate, `runs`
    times each.  The same measurement with the inputs already in device
    memory tests how much of the capacity the host-to-device copies set."""
    import gc
    import threading

    rng = np.random.default_rng(4)
    dev = torch.device("cuda:0")
    pinned = [(torch.from_numpy(m.verts).pin_memory(), torch.from_numpy(m.tets).pin_memory(), m)
              for m in pool_meshes]
    device = [(v.to(dev), t.to(dev), m) for v, t, m in pinned]
    torch.cuda.synchronize()

    def draw(n):
        pick_big = rng.random(n) < 0.1
        return [int(rng.integers(512, 544)) if b else int(rng.integers(0, 512)) for b in pick_big]

    def run_stream(srv, staged, inputs, arrivals, picks):
        tickets = [None] * len(picks)
        lat = [0.0] * len(picks)
        done_t = [0.0] * len(picks)
        sub_t = np.zeros(len(picks))
        stats = {"ok": 0}

        def collector():
            for i in range(len(picks)):
                while tickets[i] is None:
                    time.sleep(5e-5)
                srv.wait(tickets[i], timeout=120)
                done_t[i] = time.perf_counter()
                _, _, st, latency = srv.result(tickets[i])
                lat[i] = latency
                stats["ok"] += st == tv.TV_OK
                srv.release(tickets[i])

        th = threading.Thread(target=collector)
        gc.collect()
        gc.disable()  # no collector pauses inside the timed stream
        th.start()
        lag = np.zeros(len(picks))
        start = time.perf_counter()
        for i, (a, k) in enumerate(zip(arrivals, picks)):
            # sleep through long gaps (releasing the interpreter lock for the
            # collector), spin through the last 0.2 ms
            while True:
                d = a - (time.perf_counter() - start)
                if d <= 0:
                    break
                if d > 3e-4:
                    time.sleep(d - 2e-4)
            v, t, m = staged[k]
            sub_t[i] = time.perf_counter() - start
            lag[i] = sub_t[i] - a
            tickets[i] = srv.submit(v, t, m.dims, m.bbox, inputs=inputs)
        th.join()
        gc.enable()
        lat = np.array(lat)
        # the server's own completion times (submission + its latency); the
        # collector thread, which shares the interpreter lock with the
        # submitting loop, may observe them later
        span = float((sub_t + lat).max())
        client_span = max(done_t) - start
        assert stats["ok"] == len(picks), f"{len(picks) - stats['ok']} requests failed"
        return lat, span, lag, client_span

    def poisson(srv, staged, inputs, rate, n):
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
        lat, span, lag, client_span = run_stream(srv, staged, inputs, arrivals, draw(n))
        return {"offered_meshes_per_s": rate, "achieved_meshes_per_s": n / span, "requests": n,
                "client_observed_meshes_per_s": n / client_span,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "submit_lag_p99_ms": float(np.percentile(lag, 99) * 1e3)}

    def measure(staged, inputs):
        res = {}
        with tv.Server(device_bytes=32 << 30, pinned_bytes=0, streams=2, max_wave_meshes=256) as srv:
            run_stream(srv, staged, inputs, np.zeros(64), draw(64))  # warm-up
            nb = min(args.requests, 4000)
            lat, span, _, _ = run_stream(srv, staged, inputs, np.zeros(nb), draw(nb))
            burst = nb / span
            res["burst_capacity_meshes_per_s"] = burst
            # sustained capacity: rising Poisson rates until the server falls behind
            probes = []
            sustained = None

            def probe(f):
                r = poisson(srv, staged, inputs, f * burst, min(args.requests, 6000))
                probes.append([round(r["offered_meshes_per_s"]), round(r["achieved_meshes_per_s"]),
                               round(r["p99_ms"], 3)])
                return r["achieved_meshes_per_s"] >= 0.97 * r["offered_meshes_per_s"]

            for f in (0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.25):
                if not probe(f):
                    break
                sustained = f * burst
            # below half the burst rate: step down until it keeps up
            for f in (0.4, 0.3, 0.2, 0.1):
                if sustained is not None:
                    break
                if probe(f):
                    sustained = f * burst
            sustained = sustained or 0.05 * burst
            res["sustained_capacity_meshes_per_s"] = sustained
            res["capacity_probes_offered_achieved_p99"] = probes
            log(f"{inputs} inputs: burst {burst:.0f}, sustained {sustained:.0f} meshes/s; probes {probes}")
            for frac in (0.5, 0.7, 0.9):
                rs = [poisson(srv, staged, inputs, frac * sustained, args.requests) for _ in range(runs)]
                agg = {"offered_meshes_per_s": frac * sustained, "requests_per_run": args.requests, "runs": runs}
                for key in ("p50_ms", "p99_ms", "achieved_meshes_per_s", "client_observed_meshes_per_s",
                            "submit_lag_p99_ms"):
                    vals = sorted(r[key] for r in rs)
                    agg[key] = vals[len(vals) // 2]
                    agg[key + "_min_max"] = [vals[0], vals[-1]]
                agg["achieved_over_offered"] = agg["achieved_meshes_per_s"] / agg["offered_meshes_per_s"]
                log(f"{inputs} inputs, lambda={frac:.1f} x sustained: {agg}")
                res[f"lambda_{frac:.1f}"] = agg
            res["server_stats"] = {k: int(v) for k, v in srv.stats().items()}
        return res

    # a short switch interval keeps the collector thread from waiting behind
    # the submitting thread for the interpreter lock
    switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-4)
    try:
        out = measure(pinned, "pinned")
        out["device_inputs"] = measure(device, "device")
    finally:
        sys.setswitchinterval(switch)
    del device
    return out


def bench_serving(args, torch, tv):
    """The serving workload as its own line (p99 at 0.9 x sustained capacity)."""
    res = serving_core(args, torch, tv, serving_pool())
    top = res["lambda_0.9"]
    out = {"metric": "p99 latency (serving, 0.9 x sustained capacity)", "value": top["p99_ms"], "unit": "ms",
           "n_gpus": 1, "steps": args.requests, "warmup": 64, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes)",
           "config": {"workload": "Poisson request stream", "mix": "90% batch distribution, 10% medium shape",
                      "pool": "512 + 32 meshes", "inputs": "pinned host memory (device inputs alongside)",
                      "streams": 2},
           "serving": res, "roofline": None,
           "roofline_note": "the served rate is set by the host-to-device copies of the requests' inputs "
                           "(compare the device-input capacity), not by a kernel",
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def bench_grids(args, torch, tv):
    """Grid consumers on the large mesh's 1024^3 grid: the timed step is one
    tv_unpack to a dense uint8 tensor (the 3D-CNN input); pooling, float32
    unpacking and bricks are timed alongside and reported as extras."""
    log("generating workload large")
    m = make_workload("large")
    dev = torch.device("cuda:0")
    v = torch.from_numpy(m.verts).to(dev)
    t = torch.from_numpy(m.tets).to(dev)
    grid, ws = tv.voxelize(v, t, m.dims, m.bbox)
    torch.cuda.synchronize()
    del ws
    nx, ny, nz = m.dims
    n = nx * ny * nz
    out = torch.empty((nx, ny, nz), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms = timed(lambda: tv.unpack(grid, m.dims, out=out), args.steps, args.warmup)
    grid_bytes = tv.grid_words(m.dims) * 4
    alg_bytes = grid_bytes + n  # read the packed grid, write one byte per voxel
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    log(f"unpack u8: {ms:.4f} ms, {achieved:.0f} GB/s")
    extras = {}
    f32 = torch.empty((nx, ny, nz), dtype=torch.float32, device=dev)
    ms32 = timed(lambda: tv.unpack(grid, m.dims, dtype=torch.float32, out=f32), 5, 1)
    extras["unpack_f32"] = {"ms": ms32, "GB_per_s": (grid_bytes + 4 * n) / (ms32 * 1e-3) / 1e9}
    del f32
    for f in (2, 4, 8):
        po = torch.empty((nx // f, ny // f, nz // f), dtype=torch.float32, device=dev)
        msp = timed(lambda: tv.pool(grid, m.dims, f, tv.POOL_FRACTION, out=po), 5, 1)
        extras[f"pool_fraction_{f}"] = {"ms": msp, "GB_per_s": (grid_bytes + po.numel() * 4) / (msp * 1e-3) / 1e9}
    msb = timed(lambda: tv.bricks(grid, m.dims), 5, 1)
    ids, _, nbr = tv.bricks(grid, m.dims)
    extras["bricks"] = {"ms_incl_count_readback": msb, "nonempty": nbr,
                        "of": int(tv.load_library().tv_brick_count_max(tv._dims(m.dims)))}
    log(f"extras {extras}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle.grids as G

        words = grid.cpu().numpy().view(np.uint32)
        # bounded sample: whole x-slabs of the grid, grown until ~cpu_seconds
        cores = 1  # numpy unpackbits runs on one thread
        slabs = 16
        while True:
            sl = words[: slabs * ny * (nz // 32)]
            t0 = time.perf_counter()
            u = G.unpack(sl, (slabs, ny, nz))
            dt = time.perf_counter() - t0
            if dt >= 0.5 * args.cpu_seconds or slabs >= nx:
                break
            slabs = min(nx, slabs * 4)
        gpu_slab = out[:slabs].cpu().numpy()
        cpu = {"value": slabs * ny * nz / dt, "unit": "voxels/s", "cores": cores, "kind": "oracle",
               "sample": f"first {slabs} of {nx} x-slabs ({dt:.2f} s wall)",
               "gpu_bit_exact_on_sample": bool(np.array_equal(u, gpu_slab))}
    res = {"metric": "voxels unpacked/s (packed grid -> dense uint8)", "value": n / (ms * 1e-3),
           "unit": "voxels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
           "data": "synthetic (grid of the seeded large mesh)",
           "config": {"workload": "grid consumers on the large mesh's 1024^3 grid", "grid": list(m.dims)},
           "roofline": {"bound": "hbm", "kernel": "k_unpack16<16>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "algorithmic_bytes_per_launch": alg_bytes},
           "extras": extras, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def bench_bricks(args, torch, tv):
    """Sparse output: the large mesh voxelized straight into bricks at
    4096^3 (a dense grid would be 8 GiB).  The timed step is one
    tv_voxelize_bricks call; the dense path at the same resolution and the
    sparse path at 2048^3 are timed alongside, and the bricks are decoded and
    compared with the dense grid word for word."""
    log("generating workload large")
    m = make_workload("large")
    dev = torch.device("cuda:0")
    v = torch.from_numpy(m.verts).to(dev)
    t = torch.from_numpy(m.tets).to(dev)
    stream = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {}
    for n in (4096, 2048):
        dims = (n, n, n)
        nb = tv.brick_count_max(dims)
        cap = 8 << 20
        index = torch.empty(nb, dtype=torch.int32, device=dev)
        pool = torch.empty((cap, 64), dtype=torch.int32, device=dev)
        ids = torch.empty(cap, dtype=torch.int32, device=dev)
        count = torch.empty(1, dtype=torch.int32, device=dev)
        ws = tv.alloc_workspace(max(tv.bricks_workspace_bytes(m.nv, m.nt, dims),
                                    tv.workspace_bytes(m.nv, m.nt, dims)), dev)

        def step():
            tv.voxelize_bricks(v, t, dims, m.bbox, cap, index=index, pool=pool, ids=ids, count=count,
                               workspace=ws, stream=stream)
        steps = args.steps if n == 4096 else 5
        ms = timed(step, steps, args.warmup)
        assert tv.fetch_status(ws) == tv.TV_OK
        idx = index.long() & 0xFFFFFFFF
        full = int((idx == 0xFFFFFFFF).sum())
        mixed = int(((idx != 0) & (idx != 0xFFFFFFFF)).sum())
        taken = int(count.item())
        # the dense path at the same resolution, and a word-for-word check
        grid = tv.alloc_grid(dims, dev)
        ms_dense = timed(lambda: tv.voxelize(v, t, dims, m.bbox, grid=grid, workspace=ws, stream=stream),
                         3 if n == 4096 else 5, 1)
        nx = ny = nz = n
        W = nz // 32
        lanes = torch.arange(64, device=dev)
        u_, v_ = lanes // 8, lanes % 8
        nby, nbz = ny // 8, nz // 32

        def positions(b):
            bx, by, bz = b // (nby * nbz), (b // nbz) % nby, b % nbz
            return (((8 * bx[:, None] + u_) * ny + (8 * by[:, None] + v_)) * W + bz[:, None]).reshape(-1)

        sid = ids[:min(taken, cap)].long() & 0xFFFFFFFF
        live = sid != 0xFFFFFFFF
        dec = torch.zeros_like(grid)
        dec[positions(torch.nonzero(idx == 0xFFFFFFFF).reshape(-1))] = -1
        dec[positions(sid[live])] = pool[:min(taken, cap)][live].reshape(-1)
        same = bool(torch.equal(dec, grid))
        del dec, grid, index, pool, ids, ws
        torch.cuda.empty_cache()
        sparse_bytes = 4 * nb + 256 * mixed
        rec = {"ms": ms, "tets_per_s": m.nt / (ms * 1e-3), "dense_path_ms": ms_dense, "bricks": nb,
               "full_bricks": full, "pooled_bricks": mixed, "slots_taken": taken,
               "sparse_bytes": sparse_bytes, "dense_bytes": nx * ny * W * 4,
               "compression": nx * ny * W * 4 / sparse_bytes, "bit_identical_to_dense": same}
        log(f"bricks {n}^3: {rec}")
        out[str(n)] = rec
    r = out["4096"]
    res = {"metric": "tets voxelized/s (sparse bricks, no dense grid)", "value": r["tets_per_s"],
           "unit": "tets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn mesh)",
           "config": {"workload": "large mesh into 8x8x32 bricks at 4096^3", "grid": [4096] * 3,
                      "tets": m.nt},
           "bricks": out}
    print(json.dumps(res), flush=True)


QUALITY_OPS_PER_TET = 6 * 60 + 20  # six dihedral angles (cross products, norms, sqrt, acos) + exact 6V


def bench_quality(args, torch, tv):
    """Mesh files and the quality report.  The timed step is one
    tv_mesh_quality call on the large mesh (snap, per-tet report with exact
    voxel coverage, grid popcount, readback); the native readers' throughput
    on a written medium mesh is reported alongside."""
    import tempfile

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from meshfiles import write_gmsh22, write_gmsh41, write_medit

    log("generating workload large")
    m = make_workload("large")
    dev = torch.device("cuda:0")
    v = torch.from_numpy(m.verts).to(dev)
    t = torch.from_numpy(m.tets).to(dev)
    grid, _ = tv.voxelize(v, t, m.dims, m.bbox)
    ws = tv.alloc_workspace(tv.load_library().tv_quality_workspace_bytes(m.nv), dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        tv.quality(v, t, m.dims, m.bbox, grid, workspace=ws)
    tv.profile_read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        rep = tv.quality(v, t, m.dims, m.bbox, grid, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    q_lat = tv.snap(v, m.bbox).cpu().numpy()
    n_nonempty, n_cols, _ = candidate_work(q_lat, m.tets, m.dims)
    ops = QUALITY_OPS_PER_TET * m.nt + SETUP_OPS_PER_TET * n_nonempty + OPS_PER_COLUMN * n_cols
    achieved = ops / (ms * 1e-3) / 1e12
    log(f"quality: {ms:.3f} ms per report; {rep}")
    # readers
    mm = make_workload("medium")
    verts = mm.qverts.astype(np.float32) / np.float32(65536.0) if mm.verts is None else mm.verts
    readers = {}
    cpu = None
    with tempfile.TemporaryDirectory() as d:
        files = {"medit": os.path.join(d, "m.mesh"), "gmsh22": os.path.join(d, "m22.msh"),
                 "gmsh41": os.path.join(d, "m41.msh")}
        write_medit(files["medit"], verts, mm.tets)
        write_gmsh22(files["gmsh22"], verts, mm.tets)
        write_gmsh41(files["gmsh41"], verts, mm.tets)
        for k, f in files.items():
            size = os.path.getsize(f)
            t0 = time.perf_counter()
            rv, rt, _, _ = tv.read_mesh(f)
            dt = time.perf_counter() - t0
            readers[k] = {"MB": size / 1e6, "s": dt, "MB_per_s": size / 1e6 / dt, "tets": int(rt.shape[0]),
                          "exact": bool(np.array_equal(rv, verts) and np.array_equal(rt, mm.tets))}
        log(f"readers {readers}")
        if not args.no_cpu_baseline:
            import oracle.meshio as M

            size = os.path.getsize(files["medit"])
            t0 = time.perf_counter()
            ov, ot, _ = M.read_mesh(files["medit"])
            dt = time.perf_counter() - t0
            cpu = {"value": size / 1e6 / dt, "unit": "MB/s (MEDIT parse)", "cores": 1, "kind": "oracle",
                   "sample": f"the medium mesh as a {size / 1e6:.0f} MB MEDIT file ({dt:.1f} s)",
                   "native_MB_per_s": readers["medit"]["MB_per_s"],
                   "identical": bool(np.array_equal(ov, verts) and np.array_equal(ot, mm.tets))}
    res = {"metric": "tets quality-checked/s", "value": m.nt / (ms * 1e-3), "unit": "tets/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes)",
           "config": {"workload": "quality report of the large mesh; readers on the medium mesh",
                      "tets": m.nt, "grid": list(m.dims)},
           "roofline": {"bound": "alu", "kernel": "k_quality", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                        "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                        "ops_per_launch": ops, "note": "timed step includes snap, popcount and readback"},
           "report": rep, "readers": readers, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


SWEEP_N = (26, 55, 119)  # 6 n^3 = 1.05e5, 9.98e5, 1.01e7 tets, all kept


def bench_sweep(args, torch, tv):
    """Table 1's shape: whole meshes of 10^5, 10^6 and 10^7 tets (n^3 Kuhn
    cells, all kept) voxelized into 256^3, timed three ways: inputs already
    in HBM; inputs in pinned host memory copied in, grid copied back
    (PCIe-inclusive, one stream); and the CPU oracle on the host cores."""
    from paper_2106_01326_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    rows = []
    for n in SWEEP_N:
        t0 = time.perf_counter()
        m = synth.make_mesh(n, 0.3, 256, "all", 0, 5000 + n)
        log(f"n={n}: {m.nt} tets generated in {time.perf_counter() - t0:.1f} s")
        v_h = torch.from_numpy(m.verts).pin_memory()
        t_h = torch.from_numpy(m.tets).pin_memory()
        v_d, t_d = v_h.to(dev), t_h.to(dev)
        grid = tv.alloc_grid(m.dims, dev)
        ws = tv.alloc_workspace(tv.workspace_bytes(m.nv, m.nt, m.dims), dev)
        grid_h = torch.empty(grid.numel(), dtype=torch.int32).pin_memory()
        steps = max(3, min(args.steps, 20))

        def device_step():
            tv.voxelize(v_d, t_d, m.dims, m.bbox, grid=grid, workspace=ws, stream=stream)

        def pcie_step():
            v_d.copy_(v_h, non_blocking=True)
            t_d.copy_(t_h, non_blocking=True)
            tv.voxelize(v_d, t_d, m.dims, m.bbox, grid=grid, workspace=ws, stream=stream)
            grid_h.copy_(grid, non_blocking=True)

        copy_stream = torch.cuda.Stream()
        # slices of about a million tets or more: below that the per-slice launch
        # sequence costs more than the copy it hides
        slices = max(1, min(8, m.nt // 1_000_000))
        ws_pipe = tv.alloc_workspace(tv.workspace_bytes(m.nv, (m.nt + slices - 1) // slices, m.dims), dev)

        def pipelined_step():
            tv.voxelize_pipelined(v_h, t_h, m.dims, m.bbox, chunks=slices, verts_dev=v_d, tets_dev=t_d,
                                  grid=grid, workspace=ws_pipe, stream=stream, copy_stream=copy_stream)
            grid_h.copy_(grid, non_blocking=True)

        res = {}
        for name, fn in (("device", device_step), ("pcie", pcie_step), ("pcie_pipelined", pipelined_step)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name] = e0.elapsed_time(e1) / steps
            if name == "device":  # stage times from a separate profiled pass
                tv.profile_read()
                tv.profile_enable(True)
                for _ in range(3):
                    fn()
                torch.cuda.synchronize()
                tv.profile_enable(False)
                stages, calls = tv.profile_read()
                vox_ms = stages.get("voxelize", 0.0) / max(calls, 1)
        in_bytes = m.verts.nbytes + m.tets.nbytes
        row = {"n": n, "tets": m.nt, "verts": m.nv, "device_ms": res["device"], "pcie_ms": res["pcie"],
               "pcie_pipelined_ms": res["pcie_pipelined"], "pipelined_slices": slices,
               "h2d_bytes": in_bytes, "d2h_bytes": grid.numel() * 4}
        if not args.no_cpu_baseline:
            import oracle

            t0 = time.perf_counter()
            want = oracle.voxelize_q(oracle.snap(m.verts, *m.bbox), m.tets, m.dims, threads=cores)
            row["cpu_oracle_ms"] = (time.perf_counter() - t0) * 1e3
            row["bit_exact"] = bool(np.array_equal(grid_h.numpy().view(np.uint32), want))
        row["roofline"] = tile_roofline(torch, tv, [(v_d, t_d, m.dims, m.bbox, False)], [m], vox_ms)
        log(f"sweep {row}")
        rows.append(row)
        del v_d, t_d, grid, ws, ws_pipe
    big = rows[-1]
    out = {"metric": "tets voxelized/s, PCIe-inclusive (pinned host inputs in, grid out)",
           "value": big["tets"] / (big["pcie_pipelined_ms"] * 1e-3), "unit": "tets/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 2, "ms_per_step": big["pcie_pipelined_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes, all tets kept)",
           "config": {"workload": "Table 1 sweep: 1e5 / 1e6 / 1e7 tets at 256^3", "grid": [256, 256, 256],
                      "cubes_per_axis": list(SWEEP_N)},
           "sweep": rows, "roofline": big["roofline"],
           "paper_table1": "RTX 3080 + i7-10700 (other hardware, context only): 1e5 tets 1.665 s CPU+GPU vs "
                           "0.503 s CPU; 1e6 2.776 s vs 2.947 s; 1e7 9.77 s vs 98.931 s",
           "cpu_baseline": None if args.no_cpu_baseline else {
               "value": big["tets"] / (big["cpu_oracle_ms"] * 1e-3), "unit": "tets/s", "cores": cores,
               "kind": "oracle", "sample": f"the whole 1e7-tet mesh ({big['cpu_oracle_ms'] / 1e3:.1f} s)"}}
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(meshes, batch, target_s):
    """The oracle on the first meshes of the batch until about target_s of
    wall time; compared bit for bit with the batched GPU grids."""
    import oracle

    cores = host_cores()
    t0 = time.perf_counter()
    n = 0
    tets = 0
    exact = True
    while n < len(meshes) and time.perf_counter() - t0 < target_s:
        m = meshes[n]
        w = oracle.voxelize_mesh(m, threads=cores)
        exact = exact and bool(np.array_equal(w, batch.grids[n].cpu().numpy().view(np.uint32)))
        tets += m.nt
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "meshes/s", "tets_per_s": tets / dt, "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {len(meshes)} meshes ({tets} tets, {dt:.1f} s wall incl. GPU readback)",
            "gpu_bit_exact_on_sample": exact}


def tune_trials(r, defaults):
    """Compact log of a tuner search: the fields each candidate changed from
    the defaults, and its milliseconds."""
    out = []
    for e in r["log"]:
        diff = {k: v for k, v in e["params"].items() if v != defaults[k]}
        out.append([",".join(f"{k}={v}" for k, v in diff.items()) or "defaults", round(e["ms"], 4)])
    return out


def bench_tune(args, torch, tv):
    """The autotuner on the large, medium and batch workloads.  Each search
    starts from the library defaults and checks every candidate's grids
    against the defaults' word for word; the line reports the large mesh's
    tuned rate and, for each workload, default and tuned times."""
    from paper_2106_01326_amd import synth, tune

    dev = torch.device("cuda:0")
    import tempfile

    # a cache of its own, so that the run neither reads nor changes the user's
    cache = os.path.join(tempfile.mkdtemp(prefix="tetvox_tune_"), "tune.json")
    res = {}
    for name in ("large", "medium"):
        log(f"generating workload {name}")
        m = make_workload(name)
        q = m.verts is None
        v = torch.from_numpy(m.qverts if q else m.verts).to(dev)
        t = torch.from_numpy(m.tets).to(dev)
        r = tune.tune_single(v, t, m.dims, None if q else m.bbox, qverts=q, reps=5, rounds=2, cache=cache)
        res[name] = {"nt": m.nt, "ms_default": r["ms_default"], "ms_tuned": r["ms_best"],
                     "speedup": r["ms_default"] / r["ms_best"], "params": r["params"], "key": r["key"],
                     "trials": tune_trials(r, tv.default_params("single"))}
        log(f"{name}: default {r['ms_default']:.4f} ms, tuned {r['ms_best']:.4f} ms with {r['params']}")
        del v, t
    log(f"generating {args.batch_meshes} batch meshes")
    meshes = batch_meshes(args.batch_meshes)
    items = [(torch.from_numpy(m.verts).to(dev), torch.from_numpy(m.tets).to(dev), m.dims, m.bbox, False)
             for m in meshes]
    r = tune.tune_batch(tv.Batch(items), reps=3, rounds=2, cache=cache)
    res["batch"] = {"meshes": len(meshes), "ms_default": r["ms_default"], "ms_tuned": r["ms_best"],
                    "speedup": r["ms_default"] / r["ms_best"], "params": r["params"], "key": r["key"],
                    "trials": tune_trials(r, tv.default_params("batch"))}
    log(f"batch: default {r['ms_default']:.4f} ms, tuned {r['ms_best']:.4f} ms with {r['params']}")
    big = res["large"]
    out = {"metric": "tets voxelized/s (autotuned launch parameters)", "value": big["nt"] / (big["ms_tuned"] * 1e-3),
           "unit": "tets/s", "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": big["ms_tuned"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes)",
           "config": {"workload": "autotuner on the large (1024^3), medium (256^3) and batch workloads",
                      "search": "coordinate search from the defaults, 2 rounds, median of 5 (3 for the batch) "
                                "calls per candidate, every candidate bit-identical to the defaults"},
           "tuned": res, "roofline": None,
           "roofline_note": "the tuned calls run the same kernels as the large line, whose roofline applies",
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large",
                    choices=["large", "medium", "small", "batch", "serving", "grids", "quality", "sweep", "bricks",
                             "tune"])
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--batch-meshes", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--with-serving", action="store_true",
                    help="large workload: also run the serving measurement in the default line")
    ap.add_argument("--no-extras", action="store_true",
                    help="large workload only: skip the batch measurement (and the serving one, "
                         "with --with-serving) that the default line carries next to the headline")
    ap.add_argument("--cache-dir", default=None,
                    help="keep the generated single-mesh workloads as .npz files here and reuse them "
                         "(for repeated profiler passes)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the workload, run one plain device copy of this many MiB so "
                         "that a hardware-counter run can scale its byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the voxelizer is a single-GPU build "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    global CACHE_DIR
    CACHE_DIR = args.cache_dir
    # every synthetic input first: nothing below may fork or spawn workers
    # once the process has touched the GPU
    pregenerate(args)

    import torch

    import paper_2106_01326_amd as tv

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    tv.load_library()
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.full((nbytes,), 7, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    if args.workload == "batch":
        return bench_batch(args, torch, tv)
    if args.workload == "serving":
        return bench_serving(args, torch, tv)
    if args.workload == "grids":
        return bench_grids(args, torch, tv)
    if args.workload == "bricks":
        return bench_bricks(args, torch, tv)
    if args.workload == "quality":
        return bench_quality(args, torch, tv)
    if args.workload == "sweep":
        return bench_sweep(args, torch, tv)
    if args.workload == "tune":
        return bench_tune(args, torch, tv)
    m = make_workload(args.workload)
    log(f"workload {args.workload}: nt={m.nt} nv={m.nv}")

    dev = torch.device("cuda:0")
    qverts = m.verts is None
    v = torch.from_numpy(m.qverts if qverts else m.verts).to(dev)
    t = torch.from_numpy(m.tets).to(dev)
    grid = tv.alloc_grid(m.dims, dev)
    ws = tv.alloc_workspace(tv.workspace_bytes(m.nv, m.nt, m.dims), dev)
    stream = torch.cuda.current_stream()

    def step():
        tv.voxelize(v, t, m.dims, m.bbox, qverts=qverts, grid=grid, workspace=ws, stream=stream)

    for _ in range(max(1, args.warmup)):  # at least one call before its status is read
        step()
    torch.cuda.synchronize()
    assert tv.fetch_status(ws) == tv.TV_OK
    log(f"warmup done ({max(1, args.warmup)} steps)")

    # the timed steps run without the stage events; the stage (kernel) times
    # come from a separate profiled pass of the same steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    tv.profile_read()  # drop anything recorded before
    tv.profile_enable(True)
    for _ in range(max(3, min(args.steps, 10))):
        step()
    torch.cuda.synchronize()
    tv.profile_enable(False)
    stages, calls = tv.profile_read()
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step; profiled stages (ms per call) "
        f"{ {k: round(v_ / max(calls, 1), 4) for k, v_ in stages.items()} }")

    q_lat = m.qverts if qverts else tv.snap(v, m.bbox).cpu().numpy()
    n_nonempty, n_cols, n_cand = candidate_work(q_lat, m.tets, m.dims)
    words = grid.cpu().numpy().view(np.uint32)
    n_set = int(np.unpackbits(words.view(np.uint8)).sum())

    vox_ms = stages.get("voxelize", 0.0) / max(calls, 1)
    ops = SETUP_OPS_PER_TET * n_nonempty + OPS_PER_COLUMN * n_cols
    achieved = ops / (vox_ms * 1e-3) / 1e12 if vox_ms > 0 else None
    roofline = {"bound": "alu", "kernel": "k_tile_voxelize", "achieved": achieved,
                "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": (achieved / VALU_PEAK_TOPS) if achieved else None,
                "traffic": traffic_from_profiles(args.workload),
                "kernel_ms": vox_ms, "ops_per_launch": ops,
                "units": {"tets_nonempty": n_nonempty, "candidate_columns": n_cols,
                          "candidate_centers": n_cand}}

    out = {"metric": "tets voxelized/s", "value": m.nt / (ms_step * 1e-3), "unit": "tets/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered Kuhn meshes)",
           "config": workload_config(args.workload, m),
           "meshes_per_s": 1e3 / ms_step, "voxels_set_per_s": n_set / (ms_step * 1e-3),
           "stage_ms": {k: v_ / max(calls, 1) for k, v_ in stages.items()},
           "roofline": roofline}

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")

        def gpu_words(sample):
            ts = torch.from_numpy(np.ascontiguousarray(sample)).to(dev)
            g2, w2 = tv.voxelize(v, ts, m.dims, m.bbox, qverts=qverts)
            torch.cuda.synchronize()
            return g2.cpu().numpy().view(np.uint32)

        out["cpu_baseline"] = cpu_baseline(m, gpu_words, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    out["valu_counters"] = valu_counters_from_profiles(args.workload, n_cols)
    del v, t, grid, ws
    if args.workload == "large" and not args.no_extras:
        # the rest of the metric: batched vs per-mesh meshes/s on the uneven
        # batch, and serving latency percentiles
        log("batch workload (1024 uneven meshes)")
        torch.cuda.empty_cache()
        b = batch_core(args, torch, tv, batch_meshes(args.batch_meshes), steps=10, warmup=2,
                       cpu=not args.no_cpu_baseline)
        out["batch"] = {k: b[k] for k in ("meshes", "tets", "ms_per_batch", "meshes_per_s", "tets_per_s",
                                          "per_mesh_loop", "batched_over_per_mesh",
                                          "bit_identical_to_per_mesh", "graph_replay", "stage_ms", "export")}
        out["batch"]["roofline_frac"] = b["roofline"]["frac"]
        if b.get("cpu_baseline"):
            out["batch"]["oracle_bit_exact_on_sample"] = b["cpu_baseline"]["gpu_bit_exact_on_sample"]
            out["batch"]["cpu_baseline"] = b["cpu_baseline"]
        if args.with_serving:
            log("serving workload (Poisson arrivals)")
            torch.cuda.empty_cache()
            sv = serving_core(args, torch, tv, serving_pool())
            out["serving"] = sv
        else:
            out["serving"] = None
            out["serving_note"] = ("not in the default line: the serving percentiles come from "
                                   "--workload serving (or --with-serving)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
