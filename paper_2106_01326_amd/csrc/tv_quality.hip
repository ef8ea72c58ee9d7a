// Mesh quality report on the device: checks of the assumptions the paper's
// voxelizer makes about its input (Section 3, "Voxelization": a large
// minimum angle, no overlapping tets, small variance), measured on the same
// lattice the voxelizer uses.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "tv.h"
#include "tv_common.h"
#include "tv_internal.h"

namespace {

using namespace tv;

constexpr int kThreads = 256;

// accumulator slots (uint64 each) in the workspace
enum : int {
    kValid = 0,
    kDegenerate,
    kInverted,
    kInvalid,
    kBelow0,  // 4 slots: min dihedral below 1, 5, 10, 20 degrees
    kCovered = kBelow0 + 4,
    kOccupied,
    kMinDihedral,  // double bits (non-negative, so ordered as integers)
    kSumMinDihedral,
    kSumVolume,
    kSumVolume2,
    kSlots
};

__constant__ double kBelowDeg[4] = {1.0, 5.0, 10.0, 20.0};

__global__ void k_quality_clear(unsigned long long *acc) {
    const int i = threadIdx.x;
    if (i < kSlots) acc[i] = 0ull;
    if (i == kMinDihedral) {
        const double inf = __builtin_huge_val();
        acc[i] = (unsigned long long)__double_as_longlong(inf);
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}

// smallest of the six dihedral angles (degrees) of tet P[0..3] (world units)
__device__ double min_dihedral_deg(const double P[4][3]) {
    constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
    constexpr int oc[6] = {2, 1, 1, 0, 0, 0}, od[6] = {3, 3, 2, 3, 2, 1};
    double best = 180.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double *a = P[ea[k]], *b = P[eb[k]], *c = P[oc[k]], *d = P[od[k]];
        const double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double u[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
        // normals of the faces (a, b, c) and (a, b, d), both taken with the edge first
        const double n1[3] = {e[1] * u[2] - e[2] * u[1], e[2] * u[0] - e[0] * u[2], e[0] * u[1] - e[1] * u[0]};
        const double n2[3] = {e[1] * w[2] - e[2] * w[1], e[2] * w[0] - e[0] * w[2], e[0] * w[1] - e[1] * w[0]};
        const double dot = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
        const double l = sqrt((n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]) *
                              (n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]));
        const double cs = fmin(1.0, fmax(-1.0, dot / l));
        best = fmin(best, acos(cs) * (180.0 / 3.14159265358979323846));
    }
    return best;
}

// One thread per tet.
__global__ void __launch_bounds__(kThreads)
    k_quality(const int32_t *__restrict__ q, int64_t nv, const int4 *__restrict__ tets, int64_t nt,
              GridGeom g, double sx, double sy, double sz, int strict,
              unsigned long long *__restrict__ acc) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    unsigned long long c[kOccupied];  // the integer counters (slots below kOccupied)
    for (int i = 0; i < kOccupied; ++i) c[i] = 0;
    double mind = __builtin_huge_val(), sum_mind = 0.0, vol = 0.0, vol2 = 0.0;
    if (t < nt) {
        const int4 T = tets[t];
        const int32_t id[4] = {T.x, T.y, T.z, T.w};
        bool ok = true;
        for (int k = 0; k < 4; ++k) ok = ok && id[k] >= 0 && (int64_t)id[k] < nv;
        int4 V[4];
        if (ok)
            for (int k = 0; k < 4; ++k) {
                V[k] = make_int4(q[3 * (int64_t)id[k]], q[3 * (int64_t)id[k] + 1], q[3 * (int64_t)id[k] + 2], 0);
                // a failed snap is INT32_MIN; lattice input must lie in the lattice range
                ok = ok && V[k].x >= kQMin && V[k].x <= kQMax && V[k].y >= kQMin && V[k].y <= kQMax &&
                     V[k].z >= kQMin && V[k].z <= kQMax;
            }
        if (!ok) {
            c[kInvalid] = 1;
        } else {
            c[kValid] = 1;
            // 6V exactly in int64 (differences < 2^17, products < 2^51)
            const int64_t b[3] = {V[1].x - V[0].x, V[1].y - V[0].y, V[1].z - V[0].z};
            const int64_t cc[3] = {V[2].x - V[0].x, V[2].y - V[0].y, V[2].z - V[0].z};
            const int64_t d[3] = {V[3].x - V[0].x, V[3].y - V[0].y, V[3].z - V[0].z};
            const int64_t six = b[0] * (cc[1] * d[2] - cc[2] * d[1]) - b[1] * (cc[0] * d[2] - cc[2] * d[0]) +
                                b[2] * (cc[0] * d[1] - cc[1] * d[0]);
            if (six == 0) {
                c[kDegenerate] = 1;
            } else {
                c[kInverted] = six < 0 ? 1 : 0;
                double P[4][3];
                for (int k = 0; k < 4; ++k) {
                    P[k][0] = (double)V[k].x * sx;
                    P[k][1] = (double)V[k].y * sy;
                    P[k][2] = (double)V[k].z * sz;
                }
                const double md = min_dihedral_deg(P);
                mind = md;
                sum_mind = md;
                for (int k = 0; k < 4; ++k) c[kBelow0 + k] = md < kBelowDeg[k] ? 1 : 0;
                vol = fabs((double)six) * (sx * sy * sz) / 6.0;
                vol2 = vol * vol;
                // voxel centers inside (the voxelizer's rule), column by column
                int32_t lo[3], hi[3];
                if (candidate_box(V[0], V[1], V[2], V[3], g, lo, hi)) {
                    const double p0[3] = {(double)((2 * lo[0] + 1) * g.half[0]),
                                          (double)((2 * lo[1] + 1) * g.half[1]),
                                          (double)((2 * lo[2] + 1) * g.half[2])};
                    Face f[4];
                    uint32_t lower;
                    if (build_faces(V[0], V[1], V[2], V[3], p0, g, strict != 0, f, lower)) {
                        const int32_t nk = hi[2] - lo[2] + 1;
                        const double nkd = (double)nk;
                        unsigned long long cov = 0;
                        for (int32_t di = 0; di <= hi[0] - lo[0]; ++di)
                            for (int32_t dj = 0; dj <= hi[1] - lo[1]; ++dj) {
                                int32_t zl = 0, zh = nk;
                                for (int fi = 0; fi < 4; ++fi) {
                                    const double a = fma(f[fi].SY, (double)dj, fma(f[fi].SX, (double)di, f[fi].A));
                                    const int32_t th = face_threshold(f[fi], a, nkd);
                                    if ((lower >> fi) & 1u) zl = max(zl, th);
                                    else zh = min(zh, th);
                                }
                                cov += zh > zl ? (unsigned long long)(zh - zl) : 0ull;
                            }
                        c[kCovered] = cov;
                    }
                }
            }
        }
    }
    // block reduction: waves, then LDS, then one set of atomics per block
    __shared__ unsigned long long s_c[kThreads / 64][kOccupied];
    __shared__ double s_d[kThreads / 64][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = 0; i < kOccupied; ++i) {
        const unsigned long long r = wave_sum(c[i]);
        if (lane == 0) s_c[wv][i] = r;
    }
    const double r0 = wave_min(mind), r1 = wave_sum(sum_mind), r2 = wave_sum(vol), r3 = wave_sum(vol2);
    if (lane == 0) {
        s_d[wv][0] = r0;
        s_d[wv][1] = r1;
        s_d[wv][2] = r2;
        s_d[wv][3] = r3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < kOccupied; ++i) {
            unsigned long long s = 0;
            for (int w = 0; w < kThreads / 64; ++w) s += s_c[w][i];
            if (s) atomicAdd(acc + i, s);
        }
        double m = s_d[0][0], a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            m = fmin(m, s_d[w][0]);
            a1 += s_d[w][1];
            a2 += s_d[w][2];
            a3 += s_d[w][3];
        }
        if (m < __builtin_huge_val())
            atomicMin(acc + kMinDihedral, (unsigned long long)__double_as_longlong(m));
        atomicAdd(reinterpret_cast<double *>(acc + kSumMinDihedral), a1);
        atomicAdd(reinterpret_cast<double *>(acc + kSumVolume), a2);
        atomicAdd(reinterpret_cast<double *>(acc + kSumVolume2), a3);
    }
}

// Set bits of the grid: 16-byte loads (grids from the library are 256-byte
// aligned) with a word-wise tail.
__global__ void __launch_bounds__(kThreads)
    k_popcount(const uint32_t *__restrict__ grid, int64_t n, unsigned long long *__restrict__ acc) {
    unsigned long long s = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(grid) & 15u) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    const uint4 *g4 = reinterpret_cast<const uint4 *>(grid);
    for (int64_t i = t0; i < n4; i += stride) {
        const uint4 w = g4[i];
        s += (unsigned long long)(__popc(w.x) + __popc(w.y) + __popc(w.z) + __popc(w.w));
    }
    for (int64_t i = 4 * n4 + t0; i < n; i += stride) s += (unsigned long long)__popc(grid[i]);
    // one atomic per block (the counter is a single contended address)
    __shared__ unsigned long long s_w[kThreads / 64];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
        if (t) atomicAdd(acc + kOccupied, t);
    }
}

bool pow2_dim(int32_t n) { return n >= 1 && n <= 32768 && (n & (n - 1)) == 0; }

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t tv_quality_workspace_bytes(int64_t nv) {
    return nv < 0 ? 0 : round256(sizeof(unsigned long long) * kSlots) + round256((size_t)12 * (size_t)nv);
}

tv_status tv_mesh_quality(const void *verts, uint32_t vert_format, int64_t nv, const int32_t *tets,
                          int64_t nt, tv_dims dims, tv_bbox bbox, const uint32_t *grid, uint32_t flags,
                          void *ws, size_t ws_bytes, void *stream, tv_quality *out) {
    if (!out) return tv::set_error(TV_ERR_INVALID_ARG, "null output");
    memset(out, 0, sizeof *out);
    if (!pow2_dim(dims.nx) || !pow2_dim(dims.ny) || !pow2_dim(dims.nz))
        return tv::set_error(TV_ERR_UNSUPPORTED_DIMS, "dims (%d, %d, %d)", dims.nx, dims.ny, dims.nz);
    if (nv < 0 || nt < 0 || nv > INT32_MAX || (nv && !verts) || (nt && !tets) || !grid ||
        (vert_format != TV_VERTS_F32 && vert_format != TV_VERTS_Q32) || (flags & ~TV_TIE_STRICT))
        return tv::set_error(TV_ERR_INVALID_ARG, "bad quality arguments");
    for (int a = 0; a < 3; ++a)
        if (!isfinite(bbox.lo[a]) || !isfinite(bbox.hi[a]) || !(bbox.hi[a] > bbox.lo[a]))
            return tv::set_error(TV_ERR_INVALID_ARG, "bbox axis %d: need finite lo < hi", a);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < tv_quality_workspace_bytes(nv))
        return tv::set_error(TV_ERR_WORKSPACE, "quality workspace too small or misaligned");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long *acc = static_cast<unsigned long long *>(ws);
    int32_t *q = reinterpret_cast<int32_t *>(static_cast<uint8_t *>(ws) +
                                             round256(sizeof(unsigned long long) * kSlots));
    tv::BoxD box;
    double scale[3];
    for (int a = 0; a < 3; ++a) {
        box.lo[a] = (double)bbox.lo[a];
        box.ext[a] = (double)bbox.hi[a] - (double)bbox.lo[a];
        scale[a] = box.ext[a] / 65536.0;  // world units per lattice unit
    }
    k_quality_clear<<<1, 64, 0, s>>>(acc);
    if (vert_format == TV_VERTS_F32) {
        tv::launch_snap_only(static_cast<const float *>(verts), nv, box, q, s);
    } else if (nv) {
        if (hipMemcpyAsync(q, verts, (size_t)12 * (size_t)nv, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return tv::set_error(TV_ERR_HIP, "vertex copy failed");
    }
    tv::GridGeom g;
    const int32_t n[3] = {dims.nx, dims.ny, dims.nz};
    for (int a = 0; a < 3; ++a) {
        int l = 0;
        while ((1 << l) < n[a]) ++l;
        g.n[a] = n[a];
        g.shift[a] = 16 - l;
        g.half[a] = (1 << 15) / n[a];
    }
    g.words = (dims.nz + 31) / 32;
    if (nt)
        k_quality<<<(unsigned)((nt + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            q, nv, reinterpret_cast<const int4 *>(tets), nt, g, scale[0], scale[1], scale[2],
            (flags & TV_TIE_STRICT) ? 1 : 0, acc);
    const int64_t nwords = (int64_t)dims.nx * dims.ny * g.words;
    const int64_t want = (nwords / 4 + kThreads - 1) / kThreads;
    k_popcount<<<(unsigned)(want < 1 ? 1 : (want > 2048 ? 2048 : want)), kThreads, 0, s>>>(grid, nwords, acc);
    unsigned long long h[kSlots];
    if (hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return tv::set_error(TV_ERR_HIP, "quality readback failed");
    out->tets = (int64_t)h[kValid];
    out->invalid = (int64_t)h[kInvalid];
    out->degenerate = (int64_t)h[kDegenerate];
    out->inverted = (int64_t)h[kInverted];
    for (int k = 0; k < 4; ++k) out->min_dihedral_below[k] = (int64_t)h[kBelow0 + k];
    const int64_t nd = out->tets - out->degenerate;
    double md, smd, sv, sv2;
    memcpy(&md, &h[kMinDihedral], 8);
    memcpy(&smd, &h[kSumMinDihedral], 8);
    memcpy(&sv, &h[kSumVolume], 8);
    memcpy(&sv2, &h[kSumVolume2], 8);
    out->min_dihedral_deg = nd ? md : 0.0;
    out->mean_min_dihedral_deg = nd ? smd / (double)nd : 0.0;
    out->volume_mean = nd ? sv / (double)nd : 0.0;
    const double var = nd ? fmax(0.0, sv2 / (double)nd - out->volume_mean * out->volume_mean) : 0.0;
    out->volume_cv = out->volume_mean > 0.0 ? sqrt(var) / out->volume_mean : 0.0;
    out->covered_voxels = (int64_t)h[kCovered];
    out->occupied_voxels = (int64_t)h[kOccupied];
    return TV_OK;
}

}  // extern "C"
