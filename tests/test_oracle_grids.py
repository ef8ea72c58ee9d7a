"""Pins of the grid-consumer oracle (oracle/grids.py) against things other
than itself: the voxelizer oracle's independent coverage count, and plain
per-voxel Python loops that read the packed layout bit by bit."""
import numpy as np
import pytest

from paper_2106_01326_amd import synth


def grids():
    import oracle.grids as G

    return G


def bit(words, dims, i, j, k):
    nx, ny, nz = dims
    W = (nz + 31) // 32
    return (int(words[(i * ny + j) * W + k // 32]) >> (k % 32)) & 1


def random_grid(rng, dims, density=0.3):
    nx, ny, nz = dims
    W = (nz + 31) // 32
    w = np.zeros(nx * ny * W, dtype=np.uint32)
    b = rng.random((nx, ny, nz)) < density
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                if b[i, j, k]:
                    w[(i * ny + j) * W + k // 32] |= np.uint32(1 << (k % 32))
    return w, b


DIMS = [(4, 8, 64), (8, 4, 8), (2, 2, 1), (4, 4, 32), (8, 8, 16)]


@pytest.mark.parametrize("dims", DIMS)
def test_unpack_pack_against_bit_loops(dims):
    G = grids()
    rng = np.random.default_rng(11)
    w, b = random_grid(rng, dims)
    u = G.unpack(w, dims)
    assert u.dtype == np.uint8 and u.shape == dims
    assert np.array_equal(u.astype(bool), b)
    assert np.array_equal(G.pack(u), w)  # padding bits stay 0


def test_unpack_matches_voxelizer_coverage(oracle_mod):
    """The voxelizer oracle counts coverage per voxel in its own code path;
    unpacking its words must give exactly the voxels counted at least once."""
    G = grids()
    m = synth.workload_small()
    q = oracle_mod.snap(m.verts, *m.bbox)
    words, cover = oracle_mod.voxelize_q(q, m.tets, m.dims, coverage=True)
    assert np.array_equal(G.unpack(words, m.dims), (cover > 0).astype(np.uint8))


@pytest.mark.parametrize("dims,f", [((4, 8, 64), 2), ((8, 8, 16), 4), ((8, 4, 8), 4), ((4, 4, 32), 2),
                                    ((8, 8, 32), 8)])
def test_pool_against_block_loops(dims, f):
    G = grids()
    rng = np.random.default_rng(12)
    w, _ = random_grid(rng, dims, density=0.2)
    frac = G.pool_fraction(w, dims, f)
    anyw = G.pool_any(w, dims, f)
    nx, ny, nz = dims
    dout = (nx // f, ny // f, nz // f)
    for I in range(dout[0]):
        for J in range(dout[1]):
            for K in range(dout[2]):
                c = sum(bit(w, dims, f * I + a, f * J + b_, f * K + c_)
                        for a in range(f) for b_ in range(f) for c_ in range(f))
                assert frac[I, J, K] == c / f ** 3
                assert bit(anyw, dout, I, J, K) == (1 if c else 0)
    assert anyw.size == dout[0] * dout[1] * ((dout[2] + 31) // 32)


def test_pool_identities():
    G = grids()
    dims = (8, 8, 64)
    ones = G.pack(np.ones(dims, dtype=np.uint8))
    for f in (2, 4, 8):
        assert np.all(G.pool_fraction(ones, dims, f) == 1.0)
    rng = np.random.default_rng(13)
    w, b = random_grid(rng, dims, density=0.1)
    for f in (2, 4, 8):
        assert G.pool_fraction(w, dims, f).sum() * f ** 3 == b.sum()
    # a whole 8^3 grid as one block
    w8 = G.pack(b[:, :, :8])
    assert G.pool_fraction(w8, (8, 8, 8), 8)[0, 0, 0] == b[:, :, :8].sum() / 512.0


@pytest.mark.parametrize("dims", [(8, 8, 32), (16, 8, 64), (8, 16, 64)])
def test_bricks_against_loops_and_reconstruction(dims):
    G = grids()
    nx, ny, nz = dims
    rng = np.random.default_rng(14)
    w, _ = random_grid(rng, dims, density=0.002)
    ids, bw = G.bricks(w, dims)
    nby, nbz = ny // 8, nz // 32
    want = []
    for bx in range(nx // 8):
        for by in range(nby):
            for bz in range(nbz):
                if any(bit(w, dims, 8 * bx + u, 8 * by + v, 32 * bz + k)
                       for u in range(8) for v in range(8) for k in range(32)):
                    want.append((bx * nby + by) * nbz + bz)
    assert list(ids) == want
    # scattering the bricks back reproduces the grid
    W = nz // 32
    back = np.zeros_like(w)
    for id_, ws in zip(ids, bw):
        bz = int(id_) % nbz
        by = (int(id_) // nbz) % nby
        bx = int(id_) // nbz // nby
        for u in range(8):
            for v in range(8):
                back[((8 * bx + u) * ny + 8 * by + v) * W + bz] = ws[8 * u + v]
    assert np.array_equal(back, w)


# --- batched export: every cell checked against a per-cell loop over its
# source block, plus closed forms (identity at res = dims, replication as a
# Kronecker product, the set-voxel total)

def export_cell_loop(words, dims, res, I, J, K):
    """Fraction of set voxels in the source block of output cell (I, J, K),
    read bit by bit."""
    lo, hi = [], []
    for X, n in zip((I, J, K), dims):
        if n >= res:
            f = n // res
            lo.append(X * f)
            hi.append(X * f + f)
        else:
            r = res // n
            lo.append(X // r)
            hi.append(X // r + 1)
    cnt = tot = 0
    for i in range(lo[0], hi[0]):
        for j in range(lo[1], hi[1]):
            for k in range(lo[2], hi[2]):
                cnt += bit(words, dims, i, j, k)
                tot += 1
    return cnt / tot


@pytest.mark.parametrize("res", [1, 2, 4, 8])
def test_export_batch_against_cell_loops(res):
    G = grids()
    rng = np.random.default_rng(res)
    items = [random_grid(rng, d)[0] for d in ((4, 8, 16), (8, 2, 4), (1, 1, 32), (8, 8, 8))]
    dims = [(4, 8, 16), (8, 2, 4), (1, 1, 32), (8, 8, 8)]
    frac = G.export_batch(list(zip(items, dims)), res, 0)
    anyv = G.export_batch(list(zip(items, dims)), res, 1)
    assert frac.shape == anyv.shape == (4, res, res, res)
    for b, (w, d) in enumerate(zip(items, dims)):
        for I in range(res):
            for J in range(res):
                for K in range(res):
                    want = export_cell_loop(w, d, res, I, J, K)
                    assert frac[b, I, J, K] == want
                    assert anyv[b, I, J, K] == (1 if want > 0 else 0)


def test_export_batch_closed_forms():
    G = grids()
    rng = np.random.default_rng(7)
    w, bits = random_grid(rng, (8, 8, 8), 0.4)
    # at the grid's own resolution the export is the unpacked grid
    assert np.array_equal(G.export_batch([(w, (8, 8, 8))], 8, 0)[0], bits.astype(float))
    # twice as fine: every voxel becomes a 2x2x2 block of itself
    up = G.export_batch([(w, (8, 8, 8))], 16, 1)[0]
    assert np.array_equal(up, np.kron(bits.astype(np.uint8), np.ones((2, 2, 2), dtype=np.uint8)))
    # pooled: fractions times the block volume add up to the set voxels
    down = G.export_batch([(w, (8, 8, 8))], 2, 0)[0]
    assert down.sum() * 64 == bits.sum()
    # a checkerboard pooled by 2 is one half everywhere
    i, j, k = np.indices((8, 8, 8))
    cb = ((i + j + k) % 2).astype(np.uint8)
    assert np.all(G.export_batch([(G.pack(cb), (8, 8, 8))], 4, 0) == 0.5)
