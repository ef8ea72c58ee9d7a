// Device kernels of the voxelizer: ingest (snap / range check), binning of
// tets into grid tiles, the tile voxelization kernel, the large-tet kernel
// and the per-tet reference kernel.  Every kernel serves one mesh or a batch
// of meshes of uneven size in the same launch (a MeshTable maps global
// vertex, tet and tile indices to their mesh).
//
// Work decomposition.  Each grid is cut into tiles of 2^lx x 2^ly columns and
// 2^lw words (32 * 2^lw voxels) of each column.  A tet meets the tiles that
// its candidate box (the voxel centers inside its bounding box, Section 3
// "Voxelization") overlaps; each (tet, tile) pair is a "piece".  Pieces are
// counting-sorted by tile, and each tile's piece list is cut into chunks.
// One workgroup takes one chunk: it builds the chunk's pieces' face data in
// LDS, keeps per row only the columns the tet's xy projection can reach,
// splits those columns into fixed-length strips so that all lanes get equal
// work, decides every column's z span exactly and ORs it into a tile bitmap
// in LDS.  A tile covered by one chunk is then written out with plain stores
// (zeros included, so grids need no separate clear); a tile covered by
// several chunks was zeroed beforehand and each chunk ORs its non-zero words
// into it.  Tets whose candidate box meets more tiles than a fixed cap are
// set aside and handled by a separate kernel that spreads one tet's columns
// over a whole workgroup and ORs into the grid.
#include "tv_common.h"
#include "tv_kernels.h"

namespace tv {

// --------------------------------------------------------- mesh lookup

// Last m in [0, n) with pre[m] <= x (pre is non-decreasing, pre[0] = 0).
__device__ __forceinline__ int32_t find_mesh(const int64_t *__restrict__ pre, int32_t n,
                                             int64_t x) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ const MeshDesc &mesh_desc(const MeshTable &T, int32_t m) {
    return T.descs ? T.descs[m] : T.one;
}

// Meshes of the global indices [first, last] of one workgroup: threads 0 and
// 1 search the bounds once (every thread must call this), then
// mesh_in_bracket finds each index's mesh inside the bracket (usually a
// single mesh, so no search at all).
__device__ __forceinline__ void mesh_bracket(const MeshTable &T, const int64_t *pre, int64_t first,
                                             int64_t last, int32_t *s_bracket) {
    if (T.n == 1) return;
    if (threadIdx.x == 0) s_bracket[0] = find_mesh(pre, T.n, first);
    if (threadIdx.x == 1) s_bracket[1] = find_mesh(pre, T.n, last);
    __syncthreads();
}

__device__ __forceinline__ int32_t mesh_in_bracket(const MeshTable &T, const int64_t *pre, int64_t x,
                                                   const int32_t *s_bracket) {
    if (T.n == 1) return 0;
    int32_t lo = s_bracket[0], hi = s_bracket[1] + 1;  // pre[lo] <= x < pre[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ----------------------------------------------------------------- ingest

// fp32 world coordinate -> lattice coordinate, per the snap contract:
// rint(((double)v - lo) * 65536 / (hi - lo)) evaluated left to right in IEEE
// double (this file is built with -ffp-contract=off, and a subtraction
// followed by a multiplication cannot be fused anyway).  Returns false for a
// NaN or an off-range result.
__device__ __forceinline__ bool snap_coord(float v, double lo, double ext, int32_t &q) {
    double t = (double)v - lo;
    t = t * 65536.0;
    t = t / ext;
    const double r = rint(t);
    const bool in = (r >= (double)kQMin) && (r <= (double)kQMax);  // false for NaN
    q = in ? (int32_t)r : 0;
    return in;
}

// Every vertex of every mesh of the call -> padded int4 lattice record; the
// .w lane marks a vertex that is NaN or off the lattice range (such vertices
// void their tets and raise the mesh's status).
__global__ void k_ingest(MeshTable T, BinBuffers b) {
    __shared__ int32_t s_bracket[2];
    const int64_t first = (int64_t)blockIdx.x * blockDim.x;
    const int64_t last = min(first + (int64_t)blockDim.x, T.nv_total) - 1;
    const int64_t v = first + threadIdx.x;
    mesh_bracket(T, T.vert_pre, first, last, s_bracket);
    const int32_t m = mesh_in_bracket(T, T.vert_pre, min(v, last), s_bracket);
    if (v >= T.nv_total) return;
    const MeshDesc &d = mesh_desc(T, m);
    const int64_t i = v - d.vert_base;
    int32_t q[3];
    bool ok = true;
    if (d.fmt == kFmtF32) {
        const float *vf = static_cast<const float *>(d.verts);
#pragma unroll
        for (int a = 0; a < 3; ++a) ok = snap_coord(vf[3 * i + a], d.box.lo[a], d.box.ext[a], q[a]) && ok;
    } else {
        const int32_t *vq = static_cast<const int32_t *>(d.verts);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = vq[3 * i + a];
            ok = ok && q[a] >= kQMin && q[a] <= kQMax;
        }
    }
    b.q4[v] = make_int4(q[0], q[1], q[2], ok ? 0 : 1);
    if (!ok) atomicOr(b.status + d.mesh, kStatusRange);
}

// Snap into a plain [nv][3] int32 array (INT32_MIN marks a bad vertex).
__global__ void k_snap_only(const float *__restrict__ v, int64_t nv, BoxD box,
                            int32_t *__restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int32_t c[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = snap_coord(v[3 * i + a], box.lo[a], box.ext[a], c[a]) && ok;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[3 * i + a] = ok ? c[a] : INT32_MIN;
}

// Zero `n` words at `p` (4-byte aligned) with 16-byte stores where possible.
__global__ void k_clear(uint32_t *__restrict__ p, int64_t n) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t mis = (int64_t)(((uintptr_t)p >> 2) & 3);
    const int64_t head = mis ? (4 - mis < n ? 4 - mis : n) : 0;
    if (tid < head) p[tid] = 0u;
    uint4 *p4 = reinterpret_cast<uint4 *>(p + head);
    const int64_t n4 = (n - head) >> 2;
    for (int64_t i = tid; i < n4; i += stride) p4[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t tail0 = head + (n4 << 2);
    if (tid < n - tail0) p[tail0 + tid] = 0u;
}

__global__ void k_set_word(uint32_t *p, uint32_t value) { *p = value; }

// ------------------------------------------------------------- tet gather

// Six times the signed volume (Lemma 1.1), exact in double (see tv_common.h).
__device__ __forceinline__ double six_volume(const int4 V[4]) {
    const double ax = V[1].x - V[0].x, ay = V[1].y - V[0].y, az = V[1].z - V[0].z;
    const double bx = V[2].x - V[0].x, by = V[2].y - V[0].y, bz = V[2].z - V[0].z;
    const double cx = V[3].x - V[0].x, cy = V[3].y - V[0].y, cz = V[3].z - V[0].z;
    return ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
}

// Gathers the vertices of local tet `tl` of mesh d; false for a bad index
// (flagged in the mesh's status word when `status` is not null) and for a
// vertex that failed ingest (flagged there).
__device__ __forceinline__ bool gather_tet(const MeshDesc &d, const int4 *__restrict__ q4,
                                           int64_t tl, uint32_t *status, int4 V[4]) {
    const int4 T = d.tets[tl];
    if (!index_ok(T.x, d.nv) || !index_ok(T.y, d.nv) || !index_ok(T.z, d.nv) ||
        !index_ok(T.w, d.nv)) {
        if (status) atomicOr(status + d.mesh, kStatusIndex);
        return false;
    }
    const int4 *q = q4 + d.vert_base;
    V[0] = q[T.x];
    V[1] = q[T.y];
    V[2] = q[T.z];
    V[3] = q[T.w];
    return (V[0].w | V[1].w | V[2].w | V[3].w) == 0;
}

struct TileRange {
    int32_t x0, x1, y0, y1, z0, z1;  // inclusive tile index ranges
};

__device__ __forceinline__ TileRange tile_range(const int32_t lo[3], const int32_t hi[3],
                                                const TilePlan &p) {
    TileRange r;
    r.x0 = lo[0] >> p.lx;
    r.x1 = hi[0] >> p.lx;
    r.y0 = lo[1] >> p.ly;
    r.y1 = hi[1] >> p.ly;
    r.z0 = lo[2] >> (5 + p.lw);
    r.z1 = hi[2] >> (5 + p.lw);
    return r;
}

__device__ __forceinline__ uint32_t tile_id(int32_t x, int32_t y, int32_t z, const TilePlan &p) {
    return ((uint32_t)x * p.nty + y) * p.ntz + z;
}

// Shared front of both binning passes: the tet's tile range and piece
// count (0 when it contributes nothing).
__device__ __forceinline__ int32_t tet_pieces(const MeshDesc &d, const int4 *__restrict__ q4,
                                              int64_t tl, uint32_t *status, TileRange &r) {
    int4 V[4];
    if (!gather_tet(d, q4, tl, status, V)) return 0;
    int32_t lo[3], hi[3];
    if (!candidate_box(V[0], V[1], V[2], V[3], d.g, lo, hi)) return 0;
    if (six_volume(V) == 0.0) return 0;
    r = tile_range(lo, hi, d.p);
    return (r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1) * (r.z1 - r.z0 + 1);
}

// Both binning passes aggregate per workgroup: every piece's tile key goes
// into an LDS hash table (open addressing, one slot per distinct key; an
// LDS atomic counts the piece, and in pass 2 gives it its rank among the
// workgroup's pieces of that tile), then one global atomic per distinct key
// adds the workgroup's count (pass 1) or reserves its slot range (pass 2).  Neighbouring tets,
// which mostly share tiles, thus cost one global atomic per workgroup and
// tile instead of one per piece.  A key that finds no free slot within
// kHashProbes probes (a workgroup meeting very many tiles, e.g. shuffled
// tets) takes its own global atomic instead, so the table never has to
// hold every key.  The counting pass leaves a per-tet summary (first tile
// key and the tile range's shape), so the scatter pass reads 8 bytes per tet
// instead of gathering and boxing the tet again.
constexpr int kBinThreads = 256;
// tets per thread: 4 once a call has enough tets to fill the chip with
// 1024-tet workgroups (kBinTetsMany), else 2
constexpr int64_t kBinTetsMany = (int64_t)1 << 21;
constexpr int kHashSlots = 512;
constexpr int kHashProbes = 32;
constexpr int kPieceCapMax = 8;
// sparse-output calls: up to 3 x 3 x 3 tiles per tet go through the tile
// pipeline (at 4096^3 a tet of the 128^3-cube mesh meets up to 18 tiles)
constexpr int kPieceCapBricks = 27;
constexpr uint32_t kEmptyKey = 0xffffffffu;
constexpr uint32_t kNoSlot = 0xffffffffu;

// Slot of `key` in the table, inserting it if needed; kNoSlot when the
// probe sequence is exhausted.
__device__ __forceinline__ uint32_t hash_insert(uint32_t *keys, uint32_t key) {
    uint32_t h = (key * 2654435761u) >> (32 - 9);
    for (int i = 0; i < kHashProbes; ++i) {
        // slots only go from empty to a key, so a plain read that finds the
        // key (the common case: neighbouring tets share tiles) is final
        const uint32_t cur = __hip_atomic_load(keys + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == key) return h;
        if (cur == kEmptyKey) {
            const uint32_t prev = atomicCAS(keys + h, kEmptyKey, key);
            if (prev == kEmptyKey || prev == key) return h;
        }
        h = (h + 1) & (kHashSlots - 1);
    }
    return kNoSlot;
}

// Tile summary of a tet: x (the first tile's global key) and y = 0 when the
// tet has no pieces, else 1 | (nx-1) << 1 | (ny-1) << 4 | (nz-1) << 7 for a
// tile range of nx * ny * nz <= kPieceCapMax tiles.
__device__ __forceinline__ uint2 encode_trec(uint32_t key0, const TileRange &r, int32_t np) {
    if (np == 0) return make_uint2(0u, 0u);
    return make_uint2(key0, 1u | (uint32_t)(r.x1 - r.x0) << 1 | (uint32_t)(r.y1 - r.y0) << 4 |
                                (uint32_t)(r.z1 - r.z0) << 7);
}

template <bool kScatter, int kBinTets, bool kTable, int kCap = kPieceCapMax>
__global__ void __launch_bounds__(kBinThreads) k_bin(MeshTable T, BinBuffers b) {
    __shared__ uint32_t s_key[kHashSlots];
    __shared__ uint32_t s_cnt[kHashSlots];  // count, then (pass 2) global slot base
    // a batch call's pieces past the first kRef of a tet take their own
    // global atomic (a smaller table here lets more workgroups share a CU)
    constexpr int kRef = (kCap == kPieceCapMax && kTable) ? 4 : kCap;
    __shared__ uint32_t s_ref[kBinTets * kBinThreads * kRef];  // slot << 16 | rank, or kNoSlot
    __shared__ int32_t s_bracket[2];
    const int tid = threadIdx.x;
    // each thread takes kBinTets tets, kBinThreads apart (coalesced): first
    // all their tile ranges (independent gathers in flight together), then
    // their pieces into the table
    const int64_t first = (int64_t)blockIdx.x * (kBinThreads * kBinTets);
    const int64_t last = min(first + (int64_t)(kBinThreads * kBinTets), T.nt_total) - 1;
    int32_t np[kBinTets], nys[kBinTets], nzs[kBinTets];
    uint32_t key0s[kBinTets], sys[kBinTets], sxs[kBinTets];
    mesh_bracket(T, T.tet_pre, first, last, s_bracket);
    if (kTable && T.n > 1 && s_bracket[0] == s_bracket[1]) {
        // a workgroup inside one single-tile grid has nothing to bin
        const MeshDesc &d0 = T.descs[s_bracket[0]];
        if (d0.direct) {
            if (!kScatter && tid == 0 && d0.tet_base == first) b.tile_count[d0.tile_base] = (uint32_t)d0.nt;
            return;
        }
    }
    for (int i = tid; i < kHashSlots; i += kBinThreads) {
        s_key[i] = kEmptyKey;
        s_cnt[i] = 0u;
    }
    // the tile summary of this thread's tet slot u (tet t of mesh d)
    auto tile_summary = [&](int u, int64_t t, const MeshDesc &d) {
        sys[u] = (uint32_t)d.p.ntz;
        sxs[u] = (uint32_t)d.p.nty * sys[u];
        if (d.direct) {
            // a single-tile grid: every tet is a piece of its one tile, in
            // tet order, so the count is the tet count and nothing is
            // scattered (the tile kernel checks these tets' indices)
            if (!kScatter && t == d.tet_base) b.tile_count[d.tile_base] = (uint32_t)d.nt;
        } else if (!kScatter) {
            TileRange r = {0, -1, 0, -1, 0, -1};
            int32_t n = tet_pieces(d, b.q4, t - d.tet_base, b.status, r);
            // (the summary holds at most 8 tiles per axis)
            if (n > T.piece_cap || r.x1 - r.x0 > 7 || r.y1 - r.y0 > 7 || r.z1 - r.z0 > 7) {
                b.big[atomicAdd(&b.meta[kMetaBig], 1u)] = (uint32_t)t;
                n = 0;
            }
            key0s[u] = (uint32_t)d.tile_base + tile_id(r.x0, r.y0, r.z0, d.p);
            b.trec[t] = encode_trec(key0s[u], r, n);
            np[u] = n;
            nys[u] = r.y1 - r.y0 + 1;
            nzs[u] = r.z1 - r.z0 + 1;
        } else {
            const uint2 rec = b.trec[t];
            if (rec.y) {
                key0s[u] = rec.x;
                const int32_t nx = (int32_t)((rec.y >> 1) & 7u) + 1;
                nys[u] = (int32_t)((rec.y >> 4) & 7u) + 1;
                nzs[u] = (int32_t)((rec.y >> 7) & 7u) + 1;
                np[u] = nx * nys[u] * nzs[u];
            }
        }
    };
#pragma unroll
    for (int u = 0; u < kBinTets; ++u) {
        np[u] = 0;
        nys[u] = nzs[u] = 1;
        key0s[u] = sys[u] = sxs[u] = 0;
    }
    if (kTable && (T.n == 1 || s_bracket[0] == s_bracket[1])) {
        // a table call whose workgroup lies in one mesh reads the descriptor
        // once, not once per tet
        const MeshDesc d = T.descs[T.n == 1 ? 0 : s_bracket[0]];
#pragma unroll
        for (int u = 0; u < kBinTets; ++u) {
            const int64_t t = first + u * kBinThreads + tid;
            if (t < T.nt_total) tile_summary(u, t, d);
        }
    } else {
#pragma unroll
        for (int u = 0; u < kBinTets; ++u) {
            const int64_t t = first + u * kBinThreads + tid;
            if (t < T.nt_total)
                tile_summary(u, t, mesh_desc(T, mesh_in_bracket(T, T.tet_pre, min(t, last), s_bracket)));
        }
    }
    __syncthreads();  // the table is clear
#pragma unroll
    for (int u = 0; u < kBinTets; ++u) {
        const int64_t t = first + u * kBinThreads + tid;
        // the tiles of the range in (x, y, z) order, z fastest, without divisions
        int32_t dy = 0, dz = 0;
        uint32_t krow = key0s[u];  // key of tile (dx, dy, 0)
        for (int32_t k = 0; k < np[u]; ++k) {
            const uint32_t key = krow + (uint32_t)dz;
            if (++dz == nzs[u]) {
                dz = 0;
                krow += sys[u];
                if (++dy == nys[u]) {
                    dy = 0;
                    krow += sxs[u] - (uint32_t)nys[u] * sys[u];
                }
            }
            const uint32_t h = (kScatter && k >= kRef) ? kNoSlot : hash_insert(s_key, key);
            if (!kScatter) {
                // counts only: the ranks are the scatter pass's business
                if (h != kNoSlot) atomicAdd(s_cnt + h, 1u);
                else atomicAdd(b.tile_count + key, 1u);
                continue;
            }
            uint32_t ref = kNoSlot;
            if (h != kNoSlot)
                ref = (h << 16) | atomicAdd(s_cnt + h, 1u);
            else
                b.pieces[b.tile_off[key] + atomicAdd(b.tile_cursor + key, 1u)] = (uint32_t)t;
            if (k < kRef) s_ref[(u * kBinThreads + tid) * kRef + k] = ref;
        }
    }
    __syncthreads();
    for (int i = tid; i < kHashSlots; i += kBinThreads) {
        const uint32_t key = s_key[i];
        if (key == kEmptyKey) continue;
        if (kScatter) s_cnt[i] = b.tile_off[key] + atomicAdd(b.tile_cursor + key, s_cnt[i]);
        else atomicAdd(b.tile_count + key, s_cnt[i]);
    }
    if (!kScatter) return;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBinTets; ++u) {
        const int64_t t = first + u * kBinThreads + tid;
        for (int32_t k = 0; k < min(np[u], kRef); ++k) {
            const uint32_t ref = s_ref[(u * kBinThreads + tid) * kRef + k];
            if (ref != kNoSlot) b.pieces[s_cnt[ref >> 16] + (ref & 0xffffu)] = (uint32_t)t;
        }
    }
}

// Work-queue layout (one workgroup of 1024 threads, any tile count):
//   tile_off[t]    first piece slot of tile t (exclusive scan in tile order);
//   tile_order[r]  the tile of rank r: tiles sorted by size class
//                  (floor(log2 pieces), larger first; empty tiles last);
//   chunk_off[r]   first chunk of the tile of rank r (scan in rank order);
//   meta[kMetaChunks] the chunk total.
// Handing out the largest tasks first keeps the persistent workgroups busy
// until the queue runs dry, instead of leaving a few large tiles for last.
// The order inside a size class is whatever the atomics give; it changes
// which workgroup does what, never the grid.
__device__ __forceinline__ uint32_t tile_chunks(uint32_t pieces, uint32_t chunk) {
    return pieces == 0 ? 1u : (pieces + chunk - 1) / chunk;
}

// Exclusive scan over the block of 1024 values (v at tid), continuing from
// *carry; returns the exclusive prefix and advances *carry by the block
// total.  s_w: 16 words of LDS.  Every thread must call it.
__device__ __forceinline__ uint32_t scan1024(uint32_t v, uint32_t *carry, uint32_t *s_w, int tid) {
    const int lane = tid & 63, wv = tid >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t before = *carry;
    for (int w = 0; w < wv; ++w) before += s_w[w];
    uint32_t total = 0;
    for (int w = 0; w < 16; ++w) total += s_w[w];
    __syncthreads();  // s_w is rewritten by the next call
    *carry += total;
    return before + inc - v;
}

__global__ void __launch_bounds__(1024) k_scan_tiles(MeshTable T, BinBuffers b) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_class[33];  // tiles per size class, then each class's next rank
    const uint32_t nt = (uint32_t)T.ntiles_total;
    const uint32_t chunk = (uint32_t)T.chunk;
    const int tid = threadIdx.x;
    if (tid < 33) s_class[tid] = 0u;
    __syncthreads();
    // piece offsets in tile order; size-class histogram
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nt; base += 1024) {
        const uint32_t i = base + tid;
        const uint32_t c = i < nt ? b.tile_count[i] : 0u;
        const uint32_t off = scan1024(c, &carry, s_w, tid);
        if (i < nt) {
            b.tile_off[i] = off;
            atomicAdd(&s_class[__clz(c)], 1u);  // class 32: empty tiles
        }
    }
    if (tid == 0) {
        b.tile_off[nt] = carry;
        uint32_t acc = 0;
        for (int k = 0; k < 33; ++k) {
            const uint32_t n = s_class[k];
            s_class[k] = acc;
            acc += n;
        }
    }
    __syncthreads();
    // ranks: tiles of larger classes first; chunk_off[r] holds the rank's
    // chunk count until the scan below turns it into an offset
    for (uint32_t i = tid; i < nt; i += 1024) {
        const uint32_t c = b.tile_count[i];
        const uint32_t r = atomicAdd(&s_class[__clz(c)], 1u);
        b.tile_order[r] = i;
        b.chunk_off[r] = tile_chunks(c, chunk);
    }
    __syncthreads();  // chunk_off is read back by other threads below
    // chunk offsets in rank order
    carry = 0;
    for (uint32_t base = 0; base < nt; base += 1024) {
        const uint32_t r = base + tid;
        const uint32_t k = r < nt ? b.chunk_off[r] : 0u;
        const uint32_t off = scan1024(k, &carry, s_w, tid);
        if (r < nt) b.chunk_off[r] = off;
    }
    if (tid == 0) {
        b.chunk_off[nt] = carry;
        b.meta[kMetaChunks] = carry;
    }
    __syncthreads();  // every chunk offset is final
    // the task table: the rank (and mesh) behind each queue task, so that a
    // workgroup takes a task with one lookup instead of a search
    for (uint32_t r = tid; r < nt; r += 1024) {
        const uint32_t t = b.tile_order[r];
        b.rank_mesh[r] = T.n == 1 ? 0u : (uint32_t)find_mesh(T.tile_pre, T.n, (int64_t)t);
        for (uint32_t c = b.chunk_off[r]; c < b.chunk_off[r + 1]; ++c) b.task_rank[c] = r;
    }
}

// Tile origin (voxel indices) of local tile `lt` of a mesh.
struct TileOrigin {
    int32_t i0, j0, k0;
};

__device__ __forceinline__ TileOrigin tile_origin(uint32_t lt, const TilePlan &p) {
    const int32_t tz = (int32_t)(lt % (uint32_t)p.ntz);
    const uint32_t txy = lt / (uint32_t)p.ntz;
    const int32_t ty = (int32_t)(txy % (uint32_t)p.nty), tx = (int32_t)(txy / (uint32_t)p.nty);
    return {tx << p.lx, ty << p.ly, tz << (p.lw + 5)};
}

// Zero the tiles that several chunks will OR into (one workgroup per tile).
__global__ void k_zero_shared_tiles(MeshTable T, BinBuffers b) {
    const uint32_t tile = blockIdx.x;
    if (tile >= (uint32_t)T.ntiles_total) return;
    if (b.tile_count[tile] <= (uint32_t)T.chunk) return;  // one chunk: plain stores
    const int32_t m = T.n == 1 ? 0 : find_mesh(T.tile_pre, T.n, (int64_t)tile);
    const MeshDesc &d = mesh_desc(T, m);
    const TileOrigin o = tile_origin(tile - (uint32_t)d.tile_base, d.p);
    const int32_t lw = d.p.lw, ly = d.p.ly;
    const int32_t nwords = (1 << (d.p.lx + ly + lw));
    for (int32_t x = threadIdx.x; x < nwords; x += blockDim.x) {
        const int32_t cl = x >> lw;
        const int64_t i = o.i0 + (cl >> ly), j = o.j0 + (cl & ((1 << ly) - 1));
        d.grid[(i * d.g.n[1] + j) * d.g.words + (o.k0 >> 5) + (x & ((1 << lw) - 1))] = 0u;
    }
}

// Global-address-space views of device arrays: loads through them are
// global (not flat) loads, which do not count against the LDS wait counter.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
#else
template <typename T>
using gptr = const T *;  // host pass: kernels are only parsed there
#endif
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)p;
}
struct alignas(16) Int4Rec {
    int32_t x, y, z, w;
};
__device__ __forceinline__ int4 load_int4(gptr<int4> base, int64_t i) {
    const Int4Rec r = ((gptr<Int4Rec>)base)[i];
    return make_int4(r.x, r.y, r.z, r.w);
}

// ------------------------------------------------------ tile voxelization

constexpr int kTileThreads = 256;                 // four waves
constexpr int kTileWaves = kTileThreads / 64;
constexpr int kMaxTileWords = 4096;               // 16 KiB of LDS bitmap
constexpr int kWaveBatch = 64;                    // pieces per wave batch (one per lane)
constexpr int kRowPool = 1024;                    // row entries per wave batch (4 KiB)

struct PieceRec {
    Face f[4];
    int16_t ci0, cj0;   // tile-local column origin of the clipped box
    int16_t ni, k0;     // row-pool entries (non-empty rows); tile-local first z index
    int16_t nk;         // z extent
    uint16_t lower;     // faces that start the span
    uint16_t row0;      // first entry of this piece's rows in the row pool
    uint16_t ncols;     // columns kept after culling (<= 1024)
};

// z span [lo, hi) (box-relative) of column (di, dj) of a box.
__device__ __forceinline__ void column_span(const Face f[4], uint32_t lower, double di, double dj,
                                            int32_t nk, double nkd, int32_t &lo, int32_t &hi) {
    lo = 0;
    hi = nk;
#pragma unroll
    for (int fi = 0; fi < 4; ++fi) {
        const double a = fma(f[fi].SY, dj, fma(f[fi].SX, di, f[fi].A));
        const int32_t t = face_threshold(f[fi], a, nkd);
        const bool isl = (lower >> fi) & 1u;
        lo = isl ? max(lo, t) : lo;
        hi = isl ? hi : min(hi, t);
    }
}

// The tet's projection onto the xy plane is a convex polygon: the hull of
// the 4 projected vertices.  Each vertex pair (a, c) with x_a != x_c spans a
// line y = m x + b; it is a lower hull edge when the other two vertices lie
// on or above it, an upper one when they lie on or below it.  For x inside
// the polygon's x range, the polygon's cross-section is then
// [max over lower lines, min over upper lines].  A line that bounds no side
// carries -inf / +inf as its intercept so that max / min ignore it.  The
// side tests are exact (products of lattice differences stay below 2^37).
struct RowHull {
    double m[6], bl[6], bu[6];
};

__device__ __forceinline__ void make_row_hull(const int4 V[4], RowHull &h) {
    constexpr int pa[6] = {0, 0, 0, 1, 1, 2}, pc[6] = {1, 2, 3, 2, 3, 3};
    constexpr int po[6] = {2, 1, 1, 0, 0, 0}, pq[6] = {3, 3, 2, 3, 2, 1};
    const double inf = __builtin_huge_val();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int4 A = V[pa[k]], C = V[pc[k]], P = V[po[k]], Q = V[pq[k]];
        const double dx = (double)(C.x - A.x), dy = (double)(C.y - A.y);
        // sign-normalised so that a positive side means "above the line"
        const double sp = dx * (double)(P.y - A.y) - dy * (double)(P.x - A.x);
        const double sq = dx * (double)(Q.y - A.y) - dy * (double)(Q.x - A.x);
        const double up = dx > 0.0 ? 1.0 : -1.0;
        const double ap = sp * up, aq = sq * up;
        const bool line = dx != 0.0;
        // slope from the hardware reciprocal refined by one Newton step
        // (relative error near 2^-51; the culling margin needs far less)
        const double r0 = __builtin_amdgcn_rcp(line ? dx : 1.0);
        const double r1 = fma(r0, fma(-(line ? dx : 1.0), r0, 1.0), r0);
        const double m = line ? dy * r1 : 0.0;
        const double b = fma(-m, (double)A.x, (double)A.y);
        h.m[k] = m;
        h.bl[k] = (line && ap >= 0.0 && aq >= 0.0) ? b : -inf;
        h.bu[k] = (line && ap <= 0.0 && aq <= 0.0) ? b : inf;
    }
}

// Columns of row x = cx (lattice, inside the tet's x range) that the tet's
// xy projection can reach, with a one-unit margin on each side (the line
// evaluation is accurate to far better than that, so the range is
// conservative); the exact span test decides every column kept.  Returns
// the inclusive index range [j0, j1] (empty when j0 > j1).
__device__ __forceinline__ void row_columns(const RowHull &h, double cx, const GridGeom &g,
                                            int32_t &j0, int32_t &j1) {
    // finite start values keep the conversions below in range
    double ylo = -1048576.0, yhi = 1048576.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        ylo = fmax(ylo, fma(h.m[k], cx, h.bl[k]));
        yhi = fmin(yhi, fma(h.m[k], cx, h.bu[k]));
    }
    // centers (2j+1)S with ylo - 1 <= (2j+1)S <= yhi + 1
    const double S = (double)g.half[1], inv = ldexp(1.0, -g.shift[1]);  // 1 / 2S
    j0 = (int32_t)ceil((ylo - 1.0 - S) * inv);
    j1 = (int32_t)floor((yhi + 1.0 - S) * inv);
}


// ------------------------------------------------------- sparse (bricks)

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Merges one brick's contribution into the sparse output; called by a whole
// wave, lane l holding word l (column (8bx+u, 8by+v) at l = u*8 + v).  A
// brick already in the pool is ORed into; a new one either becomes
// kBrickFull (every word all ones) or takes a fresh slot: the words are
// written, then the slot is published with a compare-and-swap on the index.
// A writer that loses that race gives its slot up (ids = kBrickUnused) and
// merges into the winner's.  Several writers meet a brick only when its
// tile is shared by several tasks or a large tet covers it.
__device__ void brick_merge_wave(const BrickOut &o, uint32_t id, uint32_t word, int lane,
                                 uint32_t *status) {
    if (__ballot(word != 0u) == 0ull) return;
    const bool full = __ballot(word == 0xffffffffu) == ~0ull;
    uint32_t cur = __shfl(lane == 0 ? load_agent(o.index + id) : 0u, 0);
    for (;;) {
        if (cur == kBrickFull) return;
        if (cur != 0u) {
            if (word)
                __hip_atomic_fetch_or(o.pool + (size_t)(cur - 1u) * 64u + lane, word, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        uint32_t prev = 0;
        if (full) {
            if (lane == 0) prev = atomicCAS(o.index + id, 0u, kBrickFull);
            prev = __shfl(prev, 0);
        } else {
            uint32_t slot = 0;
            if (lane == 0) slot = atomicAdd(o.count, 1u);
            slot = __shfl(slot, 0);
            if ((int64_t)slot >= o.capacity) {
                if (lane == 0) atomicOr(status, kStatusFull);
                return;
            }
            o.pool[(size_t)slot * 64u + lane] = word;
            if (lane == 0) o.ids[slot] = id;
            __threadfence();
            if (lane == 0) prev = atomicCAS(o.index + id, 0u, slot + 1u);
            prev = __shfl(prev, 0);
            if (prev != 0u && lane == 0) o.ids[slot] = kBrickUnused;
        }
        if (prev == 0u) return;
        cur = prev;
    }
}

// The bricks of a tile bitmap in LDS (tile of 2^lx x 2^ly columns, lx and
// ly >= 3, by 2^lw words; bitmap word x = (tile column << lw) + word), one
// brick per wave at a time.
__device__ void flush_tile_bricks(const BrickOut &o, const uint32_t *bits, const TilePlan &p,
                                  int32_t ti0, int32_t tj0, int32_t tk0, int lane, int wave,
                                  int nwaves, uint32_t *status) {
    const int32_t nbx = 1 << (p.lx - 3), nby = 1 << (p.ly - 3), nbz = 1 << p.lw;
    const int32_t u = lane >> 3, v = lane & 7;
    for (int32_t bi = wave; bi < nbx * nby * nbz; bi += nwaves) {
        const int32_t bzl = bi & (nbz - 1), rest = bi >> p.lw;
        const int32_t byl = rest & (nby - 1), bxl = rest >> (p.ly - 3);
        const int32_t col = ((8 * bxl + u) << p.ly) + 8 * byl + v;
        const uint32_t word = bits[(col << p.lw) + bzl];
        const uint32_t id = ((uint32_t)((ti0 >> 3) + bxl) * (uint32_t)o.nby + (uint32_t)((tj0 >> 3) + byl)) *
                                (uint32_t)o.nbz + (uint32_t)((tk0 >> 5) + bzl);
        brick_merge_wave(o, id, word, lane, status);
    }
}

// The tile kernel's flush of a tile's bricks under sparse output, where
// every tile is one task and runs before any other writer: no brick of the
// tile has been touched, so nothing is read back or raced for.  Each wave
// classifies its bricks (at most 16), reserves pool slots for its partly
// filled ones with one atomic, then stores words, ids and index entries.
__device__ void flush_fresh_tile_bricks(const BrickOut &o, const uint32_t *bits, const TilePlan &p,
                                        int32_t ti0, int32_t tj0, int32_t tk0, int lane, int wave,
                                        int nwaves, uint32_t *status) {
    const int32_t nby = 1 << (p.ly - 3), nbz = 1 << p.lw;
    const int32_t nbt = (1 << (p.lx - 3)) * nby * nbz;
    const int32_t u = lane >> 3, v = lane & 7;
    auto brick = [&](int32_t bi, uint32_t &id) {
        const int32_t bzl = bi & (nbz - 1), rest = bi >> p.lw;
        const int32_t byl = rest & (nby - 1), bxl = rest >> (p.ly - 3);
        id = ((uint32_t)((ti0 >> 3) + bxl) * (uint32_t)o.nby + (uint32_t)((tj0 >> 3) + byl)) * (uint32_t)o.nbz +
             (uint32_t)((tk0 >> 5) + bzl);
        return bits[((((8 * bxl + u) << p.ly) + 8 * byl + v) << p.lw) + bzl];
    };
    uint32_t full = 0, mixed = 0, id;
    for (int32_t bi = wave, k = 0; bi < nbt; bi += nwaves, ++k) {
        const uint32_t w = brick(bi, id);
        if (__ballot(w != 0u) == 0ull) continue;
        if (__ballot(w == 0xffffffffu) == ~0ull) full |= 1u << k;
        else mixed |= 1u << k;
    }
    uint32_t base = 0;
    if (mixed) {
        if (lane == 0) base = atomicAdd(o.count, (uint32_t)__popc(mixed));
        base = __shfl(base, 0);
    }
    for (int32_t bi = wave, k = 0; bi < nbt; bi += nwaves, ++k) {
        if (!(((full | mixed) >> k) & 1u)) continue;
        const uint32_t w = brick(bi, id);
        if ((full >> k) & 1u) {
            if (lane == 0) o.index[id] = kBrickFull;
            continue;
        }
        const uint32_t slot = base + (uint32_t)__popc(mixed & ((1u << k) - 1u));
        if ((int64_t)slot >= o.capacity) {
            if (lane == 0) atomicOr(status, kStatusFull);
            continue;
        }
        o.pool[(size_t)slot * 64u + lane] = w;
        if (lane == 0) {
            o.ids[slot] = id;
            o.index[id] = slot + 1u;
        }
    }
}

// Wave-level scans (one value per lane of a 64-lane wave).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Next range of pieces for a wave: lane 0 advances the chunk's LDS cursor,
// every lane gets the start.
__device__ __forceinline__ uint32_t grab_pieces(uint32_t *cursor, int lane) {
    uint32_t v = 0;
    if (lane == 0) v = atomicAdd(cursor, (uint32_t)kWaveBatch);
    return __shfl(v, 0);
}

// Saturating double -> int32 conversion (the hardware conversion clamps to
// [INT32_MIN, INT32_MAX]); used on integral values only.
__device__ __forceinline__ int32_t cvt_sat_i32(double x) {
    int32_t r;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// The tile kernel.  Persistent workgroups take tasks (chunks of one tile's
// pieces) from the queue, largest tiles first.  Inside a task the four waves
// work independently: each takes batches of up to 64 pieces from the task
// and runs, without workgroup barriers,
//   (1a) one lane per piece: clipped box and the four faces -> LDS record
//        (the next batch's tets and vertices are already loading);
//   (1c) one lane per piece: the rows of the tet's xy projection, only
//        non-empty rows kept, into the wave's row pool;
//   (3)  the batch's kept columns cut into strips; each lane walks a
//        contiguous block of strips, decides each column's span exactly and
//        ORs it into the tile bitmap (LDS atomics, shared by the waves).
// The tile is written out once, after the last wave is done.
__global__ void __launch_bounds__(kTileThreads)
    k_tile_voxelize(MeshTable T, BinBuffers b, int strict) {
    __shared__ uint32_t s_bits[kMaxTileWords];
    __shared__ PieceRec s_rec[kTileWaves][kWaveBatch];
    // non-empty rows: j0 (8 bits) | count (8 bits) | di (6 bits) | prefix (10 bits)
    // (one entry more per wave: the column loop reads the entry after the
    // current one unconditionally)
    __shared__ uint32_t s_row[kTileWaves][kRowPool + 1];
    __shared__ uint32_t s_soff[kTileWaves][kWaveBatch + 1];
    __shared__ uint32_t s_chunk, s_tile, s_p0, s_p1, s_shared, s_next, s_pbase;
    __shared__ int32_t s_mesh;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t strip = (uint32_t)T.strip;
    // ceil(c / strip) as one high multiply: floor(x / strip) = mulhi(x, m)
    // with m = floor((2^32 - 1) / strip) + 1 (strip >= 2), exact for
    // x < 2^32 / strip^2 (here x < 2^11: a piece's kept columns plus strip - 1)
    const uint32_t strip_m = strip > 1u ? 0xffffffffu / strip + 1u : 0u;
    const uint32_t total = b.meta[kMetaChunks];
    PieceRec *const rec = s_rec[wv];
    uint32_t *const rows = s_row[wv];
    uint32_t *const soff = s_soff[wv];

    for (;;) {
        if (tid == 0) {
            const uint32_t c = atomicAdd(&b.meta[kMetaQueue], 1u);
            s_chunk = c;
            if (c < total) {
                const uint32_t lo = b.task_rank[c];  // the rank of the task's tile
                const uint32_t k = c - b.chunk_off[lo];
                const uint32_t nchunks = b.chunk_off[lo + 1] - b.chunk_off[lo];
                const uint32_t tile = b.tile_order[lo];
                const uint32_t pb = b.tile_off[tile], pe = b.tile_off[tile + 1];
                s_tile = tile;
                s_p0 = min(pe, pb + k * (uint32_t)T.chunk);
                s_p1 = min(pe, pb + (k + 1) * (uint32_t)T.chunk);
                s_next = s_p0;
                s_pbase = pb;
                s_shared = nchunks > 1 ? 1u : 0u;
                s_mesh = (int32_t)b.rank_mesh[lo];
            }
        }
        __syncthreads();
        if (s_chunk >= total) break;
        const uint32_t tile = s_tile, p1 = s_p1;
        const MeshDesc &d = mesh_desc(T, s_mesh);
        const GridGeom g = d.g;
        const TilePlan p = d.p;
        const gptr<int4> q4 = as_global(b.q4 + d.vert_base);
        const gptr<int4> tets = as_global(d.tets);
        const gptr<uint32_t> pieces = as_global(b.pieces);
        const uint32_t tbase = (uint32_t)d.tet_base;
        // the mesh-local tet of piece slot x: binned pieces hold global tet
        // ids; a single-tile grid's pieces are its tets in order, unbinned,
        // so only there are the indices and vertices checked here
        const bool direct = d.direct != 0;
        const uint32_t pbase = s_pbase;
        const int64_t nv = d.nv;
        auto tet_of = [&](uint32_t x) -> uint32_t { return direct ? x - pbase : pieces[x] - tbase; };
        auto tet_ok = [&](int4 &Tt) {
            if (!direct) return true;
            const bool ok = index_ok(Tt.x, nv) && index_ok(Tt.y, nv) && index_ok(Tt.z, nv) && index_ok(Tt.w, nv);
            if (!ok) Tt = make_int4(0, 0, 0, 0);  // gathered, never used
            return ok;
        };
        const int32_t tw = 1 << p.lw;
        const int32_t nwords = (1 << (p.lx + p.ly)) * tw;
        for (int32_t x = tid; x < nwords; x += kTileThreads) s_bits[x] = 0u;

        const TileOrigin o = tile_origin(tile - (uint32_t)d.tile_base, p);
        const int32_t ti0 = o.i0, tj0 = o.j0, tk0 = o.k0;
        const int32_t ti1 = ti0 + (1 << p.lx) - 1, tj1 = tj0 + (1 << p.ly) - 1;
        const int32_t tk1 = min(tk0 + (tw << 5) - 1, g.n[2] - 1);
        __syncthreads();  // bitmap cleared, s_next set

        // this wave's pending pieces: [pb, rend)
        uint32_t pb = grab_pieces(&s_next, lane);
        uint32_t rend = min(pb + (uint32_t)kWaveBatch, p1);
        // vertex records of this lane's piece in the next batch; loaded ahead
        // (the piece id -> tet -> vertex chain is three dependent gathers)
        int4 Vn[4];
        bool idx_ok = true;  // the prefetched tet's indices are in range
        if (pb + lane < rend) {
            int4 Tt = load_int4(tets, tet_of(pb + lane));
            idx_ok = tet_ok(Tt);
            Vn[0] = load_int4(q4, Tt.x);
            Vn[1] = load_int4(q4, Tt.y);
            Vn[2] = load_int4(q4, Tt.z);
            Vn[3] = load_int4(q4, Tt.w);
        }
        while (pb < rend) {
            // phase 1a: one lane per piece: clipped box, faces -> record
            const uint32_t pi = pb + lane;
            int32_t lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
            int4 Vt[4];
            uint32_t nrows = 0;
            if (direct && pi < rend && !idx_ok) atomicOr(b.status + d.mesh, kStatusIndex);
            // a vertex that failed ingest voids its tets (its mesh's status
            // was raised there; binned tets were checked when binned)
            if (pi < rend && idx_ok && (!direct || (Vn[0].w | Vn[1].w | Vn[2].w | Vn[3].w) == 0)) {
                const int4 A = Vn[0], B = Vn[1], C = Vn[2], D = Vn[3];
                Vt[0] = A;
                Vt[1] = B;
                Vt[2] = C;
                Vt[3] = D;
                candidate_box(A, B, C, D, g, lo, hi);
                lo[0] = max(lo[0], ti0);
                hi[0] = min(hi[0], ti1);
                lo[1] = max(lo[1], tj0);
                hi[1] = min(hi[1], tj1);
                lo[2] = max(lo[2], tk0);
                hi[2] = min(hi[2], tk1);
                if (lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2]) {
                    const double p0d[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                                           (double)((2 * lo[1] + 1) * g.half[1]),
                                           (double)((2 * lo[2] + 1) * g.half[2])};
                    Face f[4];
                    uint32_t lower;
                    if (build_faces(A, B, C, D, p0d, g, strict != 0, f, lower)) {
                        PieceRec &R = rec[lane];
                        // faces stored lower ones first: slot 0 always starts
                        // the span and slot 3 always ends it (every tet has both)
                        const uint32_t nl = __popc(lower);
#pragma unroll
                        for (int fi = 0; fi < 4; ++fi) {
                            const uint32_t below = (1u << fi) - 1u;
                            const uint32_t slot = ((lower >> fi) & 1u)
                                                      ? __popc(lower & below)
                                                      : nl + __popc(~lower & below);
                            R.f[slot] = f[fi];
                        }
                        lower = (1u << nl) - 1u;
                        R.ci0 = (int16_t)(lo[0] - ti0);
                        R.cj0 = (int16_t)(lo[1] - tj0);
                        R.k0 = (int16_t)(lo[2] - tk0);
                        R.nk = (int16_t)(hi[2] - lo[2] + 1);
                        R.lower = (uint16_t)lower;
                        nrows = (uint32_t)(hi[0] - lo[0] + 1);
                    }
                }
            }
            // phase 1b: row-pool offsets; the batch ends before the first
            // piece whose rows no longer fit (a piece has at most 32 rows, so
            // every batch makes progress)
            const uint32_t rincl = wave_incl_scan(nrows, lane);
            const uint32_t nb = min((uint32_t)__popcll(__ballot(rincl <= (uint32_t)kRowPool)), rend - pb);
            // the next batch: the rest of this range, or a new one
            uint32_t nbeg = pb + nb, nend = rend;
            if (nbeg >= rend) {
                nbeg = grab_pieces(&s_next, lane);
                nend = min(nbeg + (uint32_t)kWaveBatch, p1);
            }
            // the next batch's tet record, then (after phase 1c) its vertices
            // (unconditional, with the index clamped to this chunk's last piece,
            // so that nothing waits for it before its use)
            const uint32_t pn = nbeg + lane;
            int4 Tn = load_int4(tets, tet_of(min(pn, p1 - 1)));
            // phase 1c: per-row column ranges of the pieces in this batch
            uint32_t nstrips = 0;
            if ((uint32_t)lane < nb && nrows) {
                PieceRec &R = rec[lane];
                const uint32_t base = rincl - nrows;
                uint32_t prefix = 0, kept = 0;
                const uint32_t bw = (uint32_t)(hi[1] - lo[1] + 1);
                if (nrows * bw <= (uint32_t)T.nocull) {
                    // a box this small loses too little to culling to pay for it
                    for (uint32_t rr = 0; rr < nrows; ++rr) {
                        rows[base + rr] = (bw << 8) | (rr << 16) | (prefix << 22);
                        prefix += bw;
                    }
                    kept = nrows;
                } else {
                    RowHull hull;
                    make_row_hull(Vt, hull);
                    for (uint32_t rr = 0; rr < nrows; ++rr) {
                        const double cx = (double)((2 * (lo[0] + (int32_t)rr) + 1) * g.half[0]);
                        int32_t j0, j1;
                        row_columns(hull, cx, g, j0, j1);
                        j0 = max(j0, lo[1]);
                        j1 = min(j1, hi[1]);
                        if (j1 >= j0) {
                            const uint32_t cnt = (uint32_t)(j1 - j0 + 1);
                            rows[base + kept] =
                                (uint32_t)(j0 - lo[1]) | (cnt << 8) | (rr << 16) | (prefix << 22);
                            ++kept;
                            prefix += cnt;
                        }
                    }
                }
                R.ni = (int16_t)kept;
                R.row0 = (uint16_t)base;
                R.ncols = (uint16_t)prefix;
                nstrips = strip > 1u ? __umulhi(prefix + strip - 1, strip_m) : prefix;
            }
            // keeps the use of the tet record (and so its wait) after phase 1c
            asm volatile("" : "+v"(Tn.x), "+v"(Tn.y), "+v"(Tn.z), "+v"(Tn.w));
            idx_ok = tet_ok(Tn);
            if (pn < nend) {
                Vn[0] = load_int4(q4, Tn.x);
                Vn[1] = load_int4(q4, Tn.y);
                Vn[2] = load_int4(q4, Tn.z);
                Vn[3] = load_int4(q4, Tn.w);
            }
            // phase 2: exclusive scan of strip counts
            const uint32_t sincl = wave_incl_scan(nstrips, lane);
            if (lane < kWaveBatch) soff[lane] = sincl - nstrips;
            const uint32_t nst = __shfl(sincl, 63);
            if (lane == 63) soff[kWaveBatch] = nst;
            // phase 3: the batch's kept columns in strips of `strip`; each lane
            // takes a contiguous block of strips, so its faces and its row
            // position carry over from one strip to the next of the same piece
            const uint32_t sb = (uint32_t)(((uint64_t)nst * (uint32_t)lane) >> 6);
            const uint32_t se = (uint32_t)(((uint64_t)nst * (uint32_t)(lane + 1)) >> 6);
            if (sb < se) {
                int32_t pc = 0, hi_r = kWaveBatch;  // soff[pc] <= sb < soff[hi_r]
                while (hi_r - pc > 1) {
                    const int32_t mid = (pc + hi_r) >> 1;
                    if (soff[mid] <= sb) pc = mid;
                    else hi_r = mid;
                }
                double fA[4], fX[4], fY[4], fS[4], fR[4];
                int32_t ml[4], nml[4], nkm[4];  // per face: lower mask, its complement, nk & mask
                int32_t k0 = 0, colb = 0, di = 0, dj = 0, jend = 0, nkr = 0;
                uint32_t ncols = 0, pfirst = 0, pend = 0, r = 0;
                bool first = true;
                for (uint32_t s = sb; s < se; ++s) {
                    if (first || s == pend) {
                        // (next) piece with strips, positioned at its first
                        // column in this lane's block
                        if (!first)
                            do ++pc;
                            while (soff[pc + 1] <= s);
                        first = false;
                        const PieceRec &R = rec[pc];
                        const int32_t nk = R.nk;
#pragma unroll
                        for (int fi = 0; fi < 4; ++fi) {
                            fA[fi] = R.f[fi].A;
                            fX[fi] = R.f[fi].SX;
                            fY[fi] = R.f[fi].SY;
                            fS[fi] = R.f[fi].S;
                            fR[fi] = (double)R.f[fi].R;
                            ml[fi] = -(int32_t)((R.lower >> fi) & 1u);
                            nml[fi] = ~ml[fi];
                            nkm[fi] = nk & ml[fi];
                        }
                        nkr = nk;
                        k0 = R.k0;
                        colb = ((int32_t)R.ci0 << p.ly) + R.cj0;
                        ncols = R.ncols;
                        pfirst = soff[pc];
                        pend = soff[pc + 1];
                        const uint32_t row0 = R.row0;
                        const uint32_t cs = (s - pfirst) * strip;
                        // row entry holding kept column cs: last entry with prefix <= cs
                        uint32_t ra = 0, rb = cs ? (uint32_t)R.ni : 1u;
                        while (rb - ra > 1) {
                            const uint32_t mid = (ra + rb) >> 1;
                            if ((rows[row0 + mid] >> 22) <= cs) ra = mid;
                            else rb = mid;
                        }
                        r = row0 + ra;
                        const uint32_t rw = rows[r];
                        di = (int32_t)((rw >> 16) & 63u);
                        dj = (int32_t)(rw & 0xffu) + (int32_t)(cs - (rw >> 22));
                        jend = (int32_t)(rw & 0xffu) + (int32_t)((rw >> 8) & 0xffu);
                    }
                    const uint32_t c0 = (s - pfirst) * strip;
                    const uint32_t c1 = min(c0 + strip, ncols);
                    for (uint32_t c = c0; c < c1; ++c) {
                        // the next row entry, read one column ahead (used only on a
                        // row change, which happens only while columns remain)
                        const uint32_t nx = rows[r + 1];
                        const double ddi = (double)di, ddj = (double)dj;
                        int32_t tl[4], tu[4];
#pragma unroll
                        for (int fi = 0; fi < 4; ++fi) {
                            // threshold: first dk with a + S dk >= 0 (see
                            // face_threshold), here without the clamp to
                            // [0, nk]: the estimate is capped at 2^30 so that
                            // the +1 cannot overflow, and the conversion
                            // saturates below.  A value below 0 or above nk
                            // acts as 0 or nk in the max / min that follow,
                            // which include 0 and nk.
                            const double a = fma(fY[fi], ddj, fma(fX[fi], ddi, fA[fi]));
                            const double e = fmin(ceil(fma(-a, fR[fi], -0.5)), 1073741824.0);
                            const int32_t t = cvt_sat_i32(e) + (fma(fS[fi], e, a) < 0.0 ? 1 : 0);
                            tl[fi] = fi == 0 ? t : fi == 3 ? 0 : (t & ml[fi]);
                            tu[fi] = fi == 3 ? t : fi == 0 ? nkr : ((t & nml[fi]) | nkm[fi]);
                        }
                        // slot 0 is a lower face, slot 3 an upper one
                        const int32_t zlo = max(max(tl[0], tl[1]), max(tl[2], 0));
                        const int32_t zhi = min(min(tu[3], tu[1]), min(tu[2], nkr));
                        if (zlo < zhi)
                            or_run_lds(s_bits + ((colb + (di << p.ly) + dj) << p.lw), k0 + zlo,
                                       k0 + zhi);
                        // advance along the row, or to the next non-empty row
                        const bool wrap = ++dj == jend;
                        r += wrap ? 1u : 0u;
                        const int32_t nj0 = (int32_t)(nx & 0xffu);
                        di = wrap ? (int32_t)((nx >> 16) & 63u) : di;
                        dj = wrap ? nj0 : dj;
                        jend = wrap ? nj0 + (int32_t)((nx >> 8) & 0xffu) : jend;
                    }
                }
            }
            pb = nbeg;
            rend = nend;
        }
        __syncthreads();  // every wave done with this task's bitmap

        if (T.bricks.index) {
            // sparse output: the tile's bricks (this task is the tile's only
            // one, and the large tets come after)
            flush_fresh_tile_bricks(T.bricks, s_bits, p, ti0, tj0, tk0, lane, wv, kTileWaves,
                                    b.status + d.mesh);
            __syncthreads();
            continue;
        }
        // flush the tile: word x of the bitmap is word (x & (tw-1)) of
        // tile-local column x >> lw
        const bool shared_tile = s_shared != 0;
        const int64_t zbase = tk0 >> 5;
        uint32_t *__restrict__ grid = d.grid;
        for (int32_t x = tid; x < nwords; x += kTileThreads) {
            const uint32_t wv_ = s_bits[x];
            const int32_t cl = x >> p.lw;
            const int64_t i = ti0 + (cl >> p.ly), j = tj0 + (cl & ((1 << p.ly) - 1));
            const int64_t gw = (i * g.n[1] + j) * g.words + zbase + (x & (tw - 1));
            if (shared_tile) {
                if (wv_) __hip_atomic_fetch_or(grid + gw, wv_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (!T.accumulate) {
                grid[gw] = wv_;
            } else if (wv_) {
                grid[gw] |= wv_;  // this chunk owns the tile within the call
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------- large tets

// One workgroup per large tet (its candidate box meets more tiles than the
// cap): the whole box's columns are spread over the workgroup and ORed into
// the grid with word atomics.  Runs after the tile kernel.
__global__ void __launch_bounds__(256) k_large_tets(MeshTable T, BinBuffers b, int strict) {
    const uint32_t nbig = b.meta[kMetaBig];
    for (uint32_t e = blockIdx.x; e < nbig; e += gridDim.x) {
        const int64_t t = b.big[e];
        const int32_t m = T.n == 1 ? 0 : find_mesh(T.tet_pre, T.n, t);
        const MeshDesc &d = mesh_desc(T, m);
        const GridGeom g = d.g;
        const int4 Tt = d.tets[t - d.tet_base];
        const int4 *q4 = b.q4 + d.vert_base;
        const int4 A = q4[Tt.x], B = q4[Tt.y], C = q4[Tt.z], D = q4[Tt.w];
        int32_t lo[3], hi[3];
        candidate_box(A, B, C, D, g, lo, hi);
        const double p0[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                              (double)((2 * lo[1] + 1) * g.half[1]),
                              (double)((2 * lo[2] + 1) * g.half[2])};
        Face f[4];
        uint32_t lower;
        if (!build_faces(A, B, C, D, p0, g, strict != 0, f, lower)) continue;
        const uint32_t nj = (uint32_t)(hi[1] - lo[1] + 1);
        const uint32_t ncols = (uint32_t)(hi[0] - lo[0] + 1) * nj;
        const int32_t nk = hi[2] - lo[2] + 1;
        const double nkd = (double)nk;
        for (uint32_t c = threadIdx.x; c < ncols; c += blockDim.x) {
            const uint32_t di = c / nj, dj = c - di * nj;
            int32_t s0, s1;
            column_span(f, lower, (double)di, (double)dj, nk, nkd, s0, s1);
            if (s0 < s1) {
                const int64_t col = (int64_t)(lo[0] + di) * g.n[1] + (lo[1] + dj);
                or_run_global(d.grid + col * g.words, lo[2] + s0, lo[2] + s1);
            }
        }
    }
}


// Large tets with sparse output: one workgroup per tet walks the tiles its
// box meets; per tile it builds the tile bitmap in LDS from the box's
// columns, then merges the tile's bricks like the tile kernel does.
__global__ void __launch_bounds__(256) k_large_tets_bricks(MeshTable T, BinBuffers b, int strict) {
    __shared__ uint32_t s_bits[kMaxTileWords];
    const uint32_t nbig = b.meta[kMetaBig];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const MeshDesc &d = T.one;
    const GridGeom g = d.g;
    const TilePlan p = d.p;
    const int32_t tw = 1 << p.lw, nwords = (1 << (p.lx + p.ly)) << p.lw;
    for (uint32_t e = blockIdx.x; e < nbig; e += gridDim.x) {
        const int4 Tt = d.tets[b.big[e] - d.tet_base];
        const int4 *q4 = b.q4 + d.vert_base;
        const int4 A = q4[Tt.x], B = q4[Tt.y], C = q4[Tt.z], D = q4[Tt.w];
        int32_t lo[3], hi[3];
        candidate_box(A, B, C, D, g, lo, hi);
        const double p0[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                              (double)((2 * lo[1] + 1) * g.half[1]),
                              (double)((2 * lo[2] + 1) * g.half[2])};
        Face f[4];
        uint32_t lower;
        if (!build_faces(A, B, C, D, p0, g, strict != 0, f, lower)) continue;
        const int32_t nk = hi[2] - lo[2] + 1;
        const double nkd = (double)nk;
        for (int32_t tx = lo[0] >> p.lx; tx <= hi[0] >> p.lx; ++tx)
            for (int32_t ty = lo[1] >> p.ly; ty <= hi[1] >> p.ly; ++ty)
                for (int32_t tz = lo[2] >> (5 + p.lw); tz <= hi[2] >> (5 + p.lw); ++tz) {
                    const int32_t ti0 = tx << p.lx, tj0 = ty << p.ly, tk0 = tz << (5 + p.lw);
                    for (int32_t x = tid; x < nwords; x += 256) s_bits[x] = 0u;
                    __syncthreads();
                    // the box's columns inside this tile, z clipped to it
                    const int32_t i0 = max(lo[0], ti0), i1 = min(hi[0], ti0 + (1 << p.lx) - 1);
                    const int32_t j0 = max(lo[1], tj0), j1 = min(hi[1], tj0 + (1 << p.ly) - 1);
                    const int32_t z0 = max(lo[2], tk0), z1 = min(hi[2], tk0 + (tw << 5) - 1);
                    const int32_t nj = j1 - j0 + 1, ncols = (i1 - i0 + 1) * nj;
                    for (int32_t c = tid; c < ncols; c += 256) {
                        const int32_t ci = i0 + c / nj, cj = j0 + c % nj;
                        int32_t s0, s1;
                        column_span(f, lower, (double)(ci - lo[0]), (double)(cj - lo[1]), nk, nkd, s0, s1);
                        s0 = max(s0 + lo[2], z0);
                        s1 = min(s1 + lo[2], z1 + 1);
                        if (s0 < s1)
                            or_run_lds(s_bits + ((((ci - ti0) << p.ly) + (cj - tj0)) << p.lw), s0 - tk0,
                                       s1 - tk0);
                    }
                    __syncthreads();
                    flush_tile_bricks(T.bricks, s_bits, p, ti0, tj0, tk0, lane, wv, 4, b.status + d.mesh);
                    __syncthreads();
                }
    }
}

// Sparse output, last pass: a published slot whose 64 words all came out
// set (contributions merged after it was taken) becomes kBrickFull, so that
// "every voxel set" has one representation.  One wave per slot.
__global__ void __launch_bounds__(256) k_bricks_canonical(BrickOut o) {
    const int lane = threadIdx.x & 63;
    const int64_t nslots = min((int64_t)*o.count, o.capacity);
    for (int64_t s = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; s < nslots;
         s += ((int64_t)gridDim.x * 256) >> 6) {
        const uint32_t id = o.ids[s];
        if (id == kBrickUnused) continue;  // the same for every lane of the wave
        const bool full = __ballot(o.pool[(size_t)s * 64u + lane] == 0xffffffffu) == ~0ull;
        if (full && lane == 0 && o.index[id] == (uint32_t)s + 1u) {
            o.index[id] = kBrickFull;
            o.ids[s] = kBrickUnused;
        }
    }
}

// ------------------------------------------------- per-tet reference path

// One lane per tet walks all columns of its candidate box and ORs each
// column's span into the grid with word atomics.  The plainest form of the
// bounding-box scan; kept as an A/B reference for the tile pipeline (the
// grid must be cleared first).
__global__ void k_voxelize_per_tet(MeshDesc d, BinBuffers b, int strict) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.nt) return;
    int4 V[4];
    if (!gather_tet(d, b.q4, t, b.status, V)) return;
    int32_t lo[3], hi[3];
    const GridGeom g = d.g;
    if (!candidate_box(V[0], V[1], V[2], V[3], g, lo, hi)) return;
    const double p0[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                          (double)((2 * lo[1] + 1) * g.half[1]),
                          (double)((2 * lo[2] + 1) * g.half[2])};
    Face f[4];
    uint32_t lower;
    if (!build_faces(V[0], V[1], V[2], V[3], p0, g, strict != 0, f, lower)) return;
    const int32_t ni = hi[0] - lo[0] + 1, nj = hi[1] - lo[1] + 1, nk = hi[2] - lo[2] + 1;
    const double nkd = (double)nk;
    for (int32_t di = 0; di < ni; ++di) {
        for (int32_t dj = 0; dj < nj; ++dj) {
            int32_t s0, s1;
            column_span(f, lower, (double)di, (double)dj, nk, nkd, s0, s1);
            if (s0 < s1) {
                const int64_t col = (int64_t)(lo[0] + di) * g.n[1] + (lo[1] + dj);
                or_run_global(d.grid + col * g.words, lo[2] + s0, lo[2] + s1);
            }
        }
    }
}

// ------------------------------------------------------- launch wrappers

namespace {
constexpr int kBlock = 256;
inline unsigned blocks_for(int64_t n, int block = kBlock) {
    return (unsigned)((n + block - 1) / block);
}
}  // namespace

void launch_ingest(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    if (T.nv_total > 0) k_ingest<<<blocks_for(T.nv_total), kBlock, 0, s>>>(T, b);
}

void launch_snap_only(const float *v, int64_t nv, const BoxD &box, int32_t *q, hipStream_t s) {
    if (nv > 0) k_snap_only<<<blocks_for(nv), kBlock, 0, s>>>(v, nv, box, q);
}

void launch_clear(uint32_t *p, int64_t nwords, hipStream_t s) {
    if (nwords <= 0) return;
    int64_t want = (nwords / 4 + kBlock - 1) / kBlock;
    if (want < 1) want = 1;
    if (want > 8192) want = 8192;
    k_clear<<<(unsigned)want, kBlock, 0, s>>>(p, nwords);
}

void launch_set_word(uint32_t *p, uint32_t value, hipStream_t s) {
    k_set_word<<<1, 1, 0, s>>>(p, value);
}

// One binning pass, instantiated for the tets per thread and for a call
// with a descriptor table (batches) or a single descriptor argument.
template <bool kScatter>
void launch_bin(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    if (T.nt_total <= 0) return;
    if (T.piece_cap > kPieceCapMax) {
        // sparse output (one mesh): one tet per thread keeps the rank table
        // of kPieceCapBricks slots per tet within LDS
        k_bin<kScatter, 1, false, kPieceCapBricks>
            <<<(unsigned)blocks_for(T.nt_total, kBinThreads), kBinThreads, 0, s>>>(T, b);
        return;
    }
    const bool many = T.nt_total >= kBinTetsMany;
    const unsigned blocks = (unsigned)blocks_for(T.nt_total, kBinThreads * (many ? 4 : 2));
    if (T.descs) {
        if (many) k_bin<kScatter, 4, true><<<blocks, kBinThreads, 0, s>>>(T, b);
        else k_bin<kScatter, 2, true><<<blocks, kBinThreads, 0, s>>>(T, b);
    } else {
        if (many) k_bin<kScatter, 4, false><<<blocks, kBinThreads, 0, s>>>(T, b);
        else k_bin<kScatter, 2, false><<<blocks, kBinThreads, 0, s>>>(T, b);
    }
}

void launch_bin_count(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    launch_bin<false>(T, b, s);
}

void launch_scan_tiles(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    k_scan_tiles<<<1, 1024, 0, s>>>(T, b);
}

void launch_bin_scatter(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    launch_bin<true>(T, b, s);
}

void launch_zero_shared_tiles(const MeshTable &T, const BinBuffers &b, hipStream_t s) {
    if (T.ntiles_total > 0)
        k_zero_shared_tiles<<<(unsigned)T.ntiles_total, kBlock, 0, s>>>(T, b);
}

void launch_tile_voxelize(const MeshTable &T, const BinBuffers &b, bool strict, int workgroups,
                          hipStream_t s) {
    k_tile_voxelize<<<(unsigned)workgroups, kTileThreads, 0, s>>>(T, b, strict ? 1 : 0);
}

void launch_large_tets(const MeshTable &T, const BinBuffers &b, bool strict, int workgroups,
                       hipStream_t s) {
    if (T.bricks.index) k_large_tets_bricks<<<(unsigned)workgroups, 256, 0, s>>>(T, b, strict ? 1 : 0);
    else k_large_tets<<<(unsigned)workgroups, 256, 0, s>>>(T, b, strict ? 1 : 0);
}

void launch_bricks_canonical(const MeshTable &T, const BinBuffers &b, int workgroups, hipStream_t s) {
    (void)b;
    k_bricks_canonical<<<(unsigned)workgroups, 256, 0, s>>>(T.bricks);
}

void launch_voxelize_per_tet(const MeshDesc &d, const BinBuffers &b, bool strict, hipStream_t s) {
    if (d.nt > 0) k_voxelize_per_tet<<<blocks_for(d.nt), kBlock, 0, s>>>(d, b, strict ? 1 : 0);
}

int tile_max_words() { return kMaxTileWords; }

}  // namespace tv
