// Shared device-side definitions of the gfx950 voxelizer library.
//
// Exactness: every quantity of the inside test is an integer.  Vertices are
// confined to the lattice range [-2^14, 2^16 + 2^14], so coordinate
// differences are at most 1.5 * 2^16 < 2^16.59, face normals (cross products
// of edge vectors) have components below 2 * (2^16.59)^2 = 2^34.17, and a
// face function n . (P - U) at any voxel center P (P in [0, 2^16] per axis,
// so |P - U| <= 1.25 * 2^16 = 2^16.33) is below 3 * 2^34.17 * 2^16.33 =
// 2^52.09 in magnitude.  Every partial sum and product below therefore stays under
// 2^53 and is exact in IEEE double, which gfx950 executes at full rate; the
// double type is used as an exact 53-bit integer carrier, never for a
// rounded quantity, except the quotient estimates that are always followed
// by an exact integer fix-up.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tv {

constexpr int kLatticeBits = 16;
constexpr int32_t kQMin = -16384;
constexpr int32_t kQMax = 65536 + 16384;

// device status bits (per mesh)
constexpr uint32_t kStatusIndex = 1u;  // tet index outside [0, nv)
constexpr uint32_t kStatusRange = 2u;  // NaN / off-lattice coordinate

struct GridGeom {
    int32_t n[3];      // voxels per axis (powers of two)
    int32_t shift[3];  // log2 of the voxel pitch 2S in lattice units
    int32_t half[3];   // S = 2^15 / n
    int32_t words;     // W = ceil(nz / 32) words per column
};

// Candidate index range of one axis: voxel centers (2i+1)S with
// lo <= (2i+1)S <= hi, clipped to [0, n-1].  The pitch 2S is a power of two,
// so floor/ceil division are arithmetic shifts (all values fit in int32).
__device__ __forceinline__ void axis_range(int32_t lo, int32_t hi, int32_t half, int32_t shift,
                                           int32_t n, int32_t &i0, int32_t &i1) {
    i0 = -((half - lo) >> shift);  // ceil((lo - S) / 2S)
    i1 = (hi - half) >> shift;     // floor((hi - S) / 2S)
    i0 = i0 < 0 ? 0 : i0;
    i1 = i1 > n - 1 ? n - 1 : i1;
}

// The half-open tie rule: a face function that is exactly zero at a center
// counts as positive iff its gradient is lexicographically positive in the
// order (z, y, x) -- the sign it takes after the push eps*ez + eps^2*ey +
// eps^3*ex.
__device__ __forceinline__ bool lex_positive(double gx, double gy, double gz) {
    return gz > 0.0 || (gz == 0.0 && (gy > 0.0 || (gy == 0.0 && gx > 0.0)));
}

// Per-face data of one tet, relative to the center of the first candidate
// voxel (i0, j0, k0).  For candidate (i0+di, j0+dj, k0+dk) the center is
// inside this face's half-space iff
//     base + sx*di + sy*dj + sz*dk >= 0
// where base already folds in the tie rule (-1 when a zero must count as
// outside).  All values are exact integers held in doubles.
struct Face {
    double base, sx, sy, sz, rinv;  // rinv = 1/|sz| (0 when sz == 0)
};

// Builds the four inward faces of tet (A,B,C,D) (lattice coordinates) for
// the candidate box whose first center is p0.  Returns false for a
// degenerate tet.  The face opposite vertex X through (U,V,W) has normal
// (V-U) x (W-U), flipped so that X lies on its positive side; its function
// n . (P - U) is |6 vol| times X's barycentric coordinate at P, i.e. the
// same affine function whose sign Theorem 1's determinant of that face
// decides.
__device__ __forceinline__ bool build_faces(const int4 &A, const int4 &B, const int4 &C,
                                            const int4 &D, const double p0[3],
                                            const GridGeom &g, bool strict, Face f[4]) {
    const double v[4][3] = {{(double)A.x, (double)A.y, (double)A.z},
                            {(double)B.x, (double)B.y, (double)B.z},
                            {(double)C.x, (double)C.y, (double)C.z},
                            {(double)D.x, (double)D.y, (double)D.z}};
    // (opposite vertex, three face vertices)
    const int tri[4][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {2, 0, 1, 3}, {3, 0, 1, 2}};
#pragma unroll
    for (int fi = 0; fi < 4; ++fi) {
        const double *X = v[tri[fi][0]], *U = v[tri[fi][1]], *V = v[tri[fi][2]],
                     *Wv = v[tri[fi][3]];
        const double e1[3] = {V[0] - U[0], V[1] - U[1], V[2] - U[2]};
        const double e2[3] = {Wv[0] - U[0], Wv[1] - U[1], Wv[2] - U[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
        const double side = n[0] * (X[0] - U[0]) + n[1] * (X[1] - U[1]) + n[2] * (X[2] - U[2]);
        if (side == 0.0) return false;
        if (side < 0.0) {
            n[0] = -n[0];
            n[1] = -n[1];
            n[2] = -n[2];
        }
        const double tie = (!strict && lex_positive(n[0], n[1], n[2])) ? 0.0 : -1.0;
        f[fi].base = n[0] * (p0[0] - U[0]) + n[1] * (p0[1] - U[1]) + n[2] * (p0[2] - U[2]) + tie;
        f[fi].sx = n[0] * (double)(2 * g.half[0]);
        f[fi].sy = n[1] * (double)(2 * g.half[1]);
        f[fi].sz = n[2] * (double)(2 * g.half[2]);
        f[fi].rinv = f[fi].sz != 0.0 ? 1.0 / fabs(f[fi].sz) : 0.0;
    }
    return true;
}

// Narrows the z span [lo, hi) (box-relative, 0 <= lo, hi <= nk) of one column
// by one face, given a = the face value at dk = 0 of this column.
//   sz > 0: keep dk >= ceil(-a / sz)         (smallest dk with a + sz dk >= 0)
//   sz < 0: keep dk <  floor(a / |sz|) + 1   (first dk with a + sz dk < 0)
//   sz = 0: keep all or nothing (sign of a)
// The quotient comes from a reciprocal estimate (relative error < 2^-51, so
// off by at most one after clamping to [0, nk]) and is corrected by exact
// evaluations of a + sz*dk at in-box dk.
__device__ __forceinline__ void clip_span(const Face &f, double a, int32_t nk, int32_t &lo,
                                          int32_t &hi) {
    if (f.sz > 0.0) {
        double e = ceil(-a * f.rinv);
        e = fmin(fmax(e, 0.0), (double)nk);
        int32_t k = (int32_t)e;
        if (k > 0 && fma(f.sz, (double)(k - 1), a) >= 0.0) k -= 1;
        else if (k < nk && fma(f.sz, (double)k, a) < 0.0) k += 1;
        lo = k > lo ? k : lo;
    } else if (f.sz < 0.0) {
        double e = floor(a * f.rinv) + 1.0;
        e = fmin(fmax(e, 0.0), (double)nk);
        int32_t k = (int32_t)e;
        if (k > 0 && fma(f.sz, (double)(k - 1), a) < 0.0) k -= 1;
        else if (k < nk && fma(f.sz, (double)k, a) >= 0.0) k += 1;
        hi = k < hi ? k : hi;
    } else if (a < 0.0) {
        hi = 0;
    }
}

// ORs the bit run [k_lo, k_hi) (global z indices, k_lo < k_hi) into one column.
__device__ __forceinline__ void or_run_global(uint32_t *col, int32_t k_lo, int32_t k_hi) {
    const int32_t w0 = k_lo >> 5, w1 = (k_hi - 1) >> 5;
    for (int32_t w = w0; w <= w1; ++w) {
        uint32_t m = 0xffffffffu;
        if (w == w0) m &= 0xffffffffu << (k_lo & 31);
        if (w == w1) m &= 0xffffffffu >> (31 - ((k_hi - 1) & 31));
        __hip_atomic_fetch_or(col + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace tv
