// Device kernels of the single-mesh path: ingest (snap / range check),
// grid clearing and the per-tet voxelization kernel.
#include "tv_common.h"
#include "tv_kernels.h"

namespace tv {

// ----------------------------------------------------------------- ingest

// fp32 world coordinates -> lattice coordinates, per the snap contract:
// rint(((double)v - lo) * 65536 / (hi - lo)) evaluated left to right in IEEE
// double (this file is built with -ffp-contract=off, and a subtraction
// followed by a multiplication cannot be fused anyway).  The .w lane marks a
// vertex that is NaN or off the lattice range; such vertices void their tets.
__global__ void k_ingest_f32(const float *__restrict__ v, int64_t nv, BoxD box,
                             int4 *__restrict__ q4, uint32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int32_t q[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = (double)v[3 * i + a] - box.lo[a];
        t = t * 65536.0;
        t = t / box.ext[a];
        const double r = rint(t);
        const bool in = (r >= (double)kQMin) && (r <= (double)kQMax);  // false for NaN
        ok = ok && in;
        q[a] = in ? (int32_t)r : 0;
    }
    q4[i] = make_int4(q[0], q[1], q[2], ok ? 0 : 1);
    if (!ok) atomicOr(status, kStatusRange);
}

// int32 lattice coordinates -> padded int4 with the same range check.
__global__ void k_ingest_q32(const int32_t *__restrict__ qin, int64_t nv, int4 *__restrict__ q4,
                             uint32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int32_t x = qin[3 * i], y = qin[3 * i + 1], z = qin[3 * i + 2];
    const bool ok = x >= kQMin && x <= kQMax && y >= kQMin && y <= kQMax && z >= kQMin &&
                    z <= kQMax;
    q4[i] = make_int4(x, y, z, ok ? 0 : 1);
    if (!ok) atomicOr(status, kStatusRange);
}

// Zero `nwords` words at `p` (any 4-byte alignment) plus `nstatus` status
// words.  A plain fill kernel rather than a memset node, so the same launch
// sequence can be captured into a graph.
__global__ void k_clear(uint32_t *__restrict__ p, int64_t nwords, uint32_t *__restrict__ st,
                        int32_t nstatus) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (tid < nstatus) st[tid] = 0u;
    // peel to 16-byte alignment
    const int64_t mis = (int64_t)(((uintptr_t)p >> 2) & 3);
    const int64_t head = mis ? (4 - mis < nwords ? 4 - mis : nwords) : 0;
    if (tid < head) p[tid] = 0u;
    uint4 *p4 = reinterpret_cast<uint4 *>(p + head);
    const int64_t n4 = (nwords - head) >> 2;
    for (int64_t i = tid; i < n4; i += stride) p4[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t tail0 = head + (n4 << 2);
    if (tid < nwords - tail0) p[tail0 + tid] = 0u;
}

// ------------------------------------------------- per-tet voxelization

// One lane per tet: gather its four lattice vertices, cull degenerate tets
// and empty candidate boxes, then walk the (x, y) columns of the candidate
// box; each column's z span comes from the four exact face bounds and is
// ORed into the grid with word-level atomics.  The simplest form of the
// bounding-box scan (Section 3, "Voxelization"); kept as an A/B reference
// for the binned kernel.
__global__ void k_voxelize_per_tet(const int4 *__restrict__ q4, int64_t nv,
                                   const int4 *__restrict__ tets, int64_t nt, GridGeom g,
                                   uint32_t *__restrict__ grid, uint32_t *__restrict__ status,
                                   int strict) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int4 T = tets[t];
    if (!index_ok(T.x, nv) || !index_ok(T.y, nv) || !index_ok(T.z, nv) || !index_ok(T.w, nv)) {
        atomicOr(status, kStatusIndex);
        return;
    }
    const int4 A = q4[T.x], B = q4[T.y], C = q4[T.z], D = q4[T.w];
    if (A.w | B.w | C.w | D.w) return;  // a vertex failed ingest (already flagged)

    int32_t lo[3], hi[3];
    const int32_t mn[3] = {min(min(A.x, B.x), min(C.x, D.x)), min(min(A.y, B.y), min(C.y, D.y)),
                           min(min(A.z, B.z), min(C.z, D.z))};
    const int32_t mx[3] = {max(max(A.x, B.x), max(C.x, D.x)), max(max(A.y, B.y), max(C.y, D.y)),
                           max(max(A.z, B.z), max(C.z, D.z))};
#pragma unroll
    for (int a = 0; a < 3; ++a) axis_range(mn[a], mx[a], g.half[a], g.shift[a], g.n[a], lo[a], hi[a]);
    if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) return;

    const double p0[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                          (double)((2 * lo[1] + 1) * g.half[1]),
                          (double)((2 * lo[2] + 1) * g.half[2])};
    Face f[4];
    if (!build_faces(A, B, C, D, p0, g, strict != 0, f)) return;

    const int32_t ni = hi[0] - lo[0] + 1, nj = hi[1] - lo[1] + 1, nk = hi[2] - lo[2] + 1;
    for (int32_t di = 0; di < ni; ++di) {
        for (int32_t dj = 0; dj < nj; ++dj) {
            int32_t klo = 0, khi = nk;
#pragma unroll
            for (int fi = 0; fi < 4; ++fi) {
                const double a = fma(f[fi].sy, (double)dj, fma(f[fi].sx, (double)di, f[fi].base));
                clip_span(f[fi], a, nk, klo, khi);
            }
            if (klo < khi) {
                const int64_t col = (int64_t)(lo[0] + di) * g.n[1] + (lo[1] + dj);
                or_run_global(grid + col * g.words, lo[2] + klo, lo[2] + khi);
            }
        }
    }
}

// ------------------------------------------------------- launch wrappers

namespace {
constexpr int kBlock = 256;
inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
}  // namespace

void launch_ingest_f32(const float *v, int64_t nv, const BoxD &box, int4 *q4, uint32_t *status,
                       hipStream_t s) {
    if (nv > 0) k_ingest_f32<<<blocks_for(nv), kBlock, 0, s>>>(v, nv, box, q4, status);
}

void launch_ingest_q32(const int32_t *q, int64_t nv, int4 *q4, uint32_t *status, hipStream_t s) {
    if (nv > 0) k_ingest_q32<<<blocks_for(nv), kBlock, 0, s>>>(q, nv, q4, status);
}

void launch_clear(uint32_t *p, int64_t nwords, uint32_t *status, int32_t nstatus, hipStream_t s) {
    int64_t want = (nwords / 4 + kBlock - 1) / kBlock;
    if (want < 1) want = 1;
    if (want > 8192) want = 8192;
    k_clear<<<(unsigned)want, kBlock, 0, s>>>(p, nwords, status, nstatus);
}

void launch_voxelize_per_tet(const int4 *q4, int64_t nv, const int4 *tets, int64_t nt,
                             const GridGeom &g, uint32_t *grid, uint32_t *status, bool strict,
                             hipStream_t s) {
    if (nt > 0)
        k_voxelize_per_tet<<<blocks_for(nt), kBlock, 0, s>>>(q4, nv, tets, nt, g, grid, status,
                                                             strict ? 1 : 0);
}

}  // namespace tv
