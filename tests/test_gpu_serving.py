"""Serving loop on the GPU: requests that arrive while others run are
admitted into later waves, waves overlap on the device, and every result is
bit-identical alone and in the mix (and to the oracle)."""
import threading
import time

import numpy as np
import pytest

from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[case] {msg}", flush=True)


def grid_of(srv, ticket, dims):
    import paper_2106_01326_amd as tv

    out = np.empty(tv.grid_words(dims), dtype=np.uint32)
    srv.copy_grid(ticket, out)
    return out


@pytest.fixture(scope="module")
def mix():
    ms = synth.workload_batch(first=36, seed=4, workers=8)
    ms += [synth.make_mesh(32, 0.3, 256, "ellipsoids", 3, 4000 + i) for i in range(2)]
    ms.append(synth.make_mesh(16, 0.2, 64, "ellipsoids", 2, 4100, fmt="q32"))
    return ms


def submit_mesh(srv, m, inputs="host", strict=False):
    if m.verts is not None:
        return srv.submit(m.verts, m.tets, m.dims, m.bbox, strict=strict, inputs=inputs)
    return srv.submit(m.qverts, m.tets, m.dims, qverts=True, strict=strict, inputs=inputs)


def test_results_alone_and_in_the_mix(oracle_mod, mix):
    import paper_2106_01326_amd as tv

    banner(f"serving mix of {len(mix)} requests")
    alone = []
    with tv.Server(device_bytes=2 << 30, pinned_bytes=256 << 20, streams=2) as srv:
        for m in mix:  # one at a time: each is a wave of its own
            t = submit_mesh(srv, m)
            srv.wait(t, timeout=60)
            _, _, st, _ = srv.result(t)
            assert st == tv.TV_OK
            alone.append(grid_of(srv, t, m.dims))
            srv.release(t)
    with tv.Server(device_bytes=2 << 30, pinned_bytes=256 << 20, streams=2, max_wave_meshes=8) as srv:
        # arrivals from two client threads with jittered gaps, so requests
        # land while earlier waves are on the device
        tickets = [None] * len(mix)
        rng = np.random.default_rng(5)
        gaps = rng.exponential(2e-4, size=len(mix))

        def client(idx):
            for i in idx:
                time.sleep(gaps[i])
                tickets[i] = submit_mesh(srv, mix[i])

        ths = [threading.Thread(target=client, args=(list(range(k, len(mix), 2)),)) for k in range(2)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        lat = []
        for i, m in enumerate(mix):
            srv.wait(tickets[i], timeout=60)
            _, words, st, latency = srv.result(tickets[i])
            assert st == tv.TV_OK and words == tv.grid_words(m.dims)
            got = grid_of(srv, tickets[i], m.dims)
            assert np.array_equal(got, alone[i]), f"request {i} differs from its solo result"
            assert np.array_equal(got, oracle_mod.voxelize_mesh(m)), f"request {i} differs from the oracle"
            lat.append(latency)
            srv.release(tickets[i])
        s = srv.stats()
        assert s["completed"] == len(mix) and s["released"] == len(mix)
        assert s["waves"] < len(mix)  # requests were batched
        assert all(x > 0 for x in lat)
        assert s["device_in_use"] == 0 and s["queued"] == 0


def test_admission_by_memory_footprint(oracle_mod, mix):
    """A small device arena: requests queue until memory frees up, the peak
    never exceeds the arena, everything completes; a request that could never
    fit is refused at submission."""
    import paper_2106_01326_amd as tv

    small = [m for m in mix if m.dims[0] <= 64][:20]
    per = max(tv.grid_words(m.dims) * 4 + m.nt * 60 + m.nv * 40 for m in small)
    arena = 4 * per + (4 << 20)
    with tv.Server(device_bytes=arena, pinned_bytes=64 << 20, streams=2, max_wave_meshes=64) as srv:
        tickets = [submit_mesh(srv, m) for m in small]
        for t, m in zip(tickets, small):
            srv.wait(t, timeout=60)
            assert np.array_equal(grid_of(srv, t, m.dims), oracle_mod.voxelize_mesh(m))
            srv.release(t)
        s = srv.stats()
        assert s["device_peak"] <= arena
        assert s["waves"] >= 2  # memory pressure split the work
        big = synth.workload_small()
        big.dims = (1024, 1024, 1024)  # a 128 MiB grid: larger than the whole arena
        assert arena < 128 << 20
        with pytest.raises(tv.TVError) as e:
            submit_mesh(srv, big)
        assert e.value.code == tv.TV_ERR_TOO_LARGE
        assert srv.stats()["rejected"] == 1


def test_input_modes_and_strict(oracle_mod, mix):
    import torch

    import paper_2106_01326_amd as tv

    ms = mix[:6]
    with tv.Server(device_bytes=1 << 30, pinned_bytes=64 << 20, streams=3) as srv:
        tickets = []
        for i, m in enumerate(ms):
            if i % 3 == 0:
                tickets.append(submit_mesh(srv, m, "host", strict=(i == 3)))
            elif i % 3 == 1:
                v = torch.from_numpy(m.verts).pin_memory()
                t = torch.from_numpy(m.tets).pin_memory()
                tickets.append(srv.submit(v, t, m.dims, m.bbox, inputs="pinned"))
            else:
                v = torch.from_numpy(m.verts).cuda()
                t = torch.from_numpy(m.tets).cuda()
                tickets.append(srv.submit(v, t, m.dims, m.bbox, inputs="device"))
        for i, (t, m) in enumerate(zip(tickets, ms)):
            srv.wait(t, timeout=60)
            mode = oracle_mod.STRICT if i == 3 else oracle_mod.HALF_OPEN
            assert np.array_equal(grid_of(srv, t, m.dims), oracle_mod.voxelize_mesh(m, mode=mode))
            srv.release(t)
        # a bad request reports its data error without disturbing others
        m = ms[0]
        bad = np.concatenate([m.tets, np.array([[0, 1, 2, m.nv + 3]], np.int32)])
        tb = srv.submit(m.verts, bad, m.dims, m.bbox)
        tg = submit_mesh(srv, ms[1])
        srv.wait(tb, timeout=60)
        srv.wait(tg, timeout=60)
        assert srv.result(tb)[2] == tv.TV_ERR_INDEX
        assert srv.result(tg)[2] == tv.TV_OK
        assert np.array_equal(grid_of(srv, tb, m.dims), oracle_mod.voxelize_mesh(m))
        with pytest.raises(tv.TVError):
            srv.release(987654)


def test_waves_overlap_on_the_device(oracle_mod, mix):
    """A long request (a 256^3 grid) followed at once by small ones, with two
    streams and small waves: a second wave is launched while the first is
    still on the device, so at least two waves are in flight together."""
    import paper_2106_01326_amd as tv

    long_req = [m for m in mix if m.dims[0] == 256][0]
    small = [m for m in mix if m.dims[0] <= 64][:24]
    with tv.Server(device_bytes=2 << 30, pinned_bytes=256 << 20, streams=2, max_wave_meshes=4) as srv:
        banner("overlap: one 256^3 request then 24 small ones")
        tickets = [submit_mesh(srv, long_req)] + [submit_mesh(srv, m) for m in small]
        for t, m in zip(tickets, [long_req] + small):
            srv.wait(t, timeout=60)
            assert srv.result(t)[2] == tv.TV_OK
            assert np.array_equal(grid_of(srv, t, m.dims), oracle_mod.voxelize_mesh(m))
            srv.release(t)
        s = srv.stats()
        assert s["waves"] >= 2
        assert s["inflight_peak"] >= 2, s
