// Shared device-side definitions of the gfx950 voxelizer library.
//
// Exactness: every quantity of the inside test is an integer.  Vertices are
// confined to the lattice range [-2^14, 2^16 + 2^14], so coordinate
// differences are at most 1.5 * 2^16 < 2^16.59, face normals (cross products
// of edge vectors) have components below 2 * (2^16.59)^2 = 2^34.17, and a
// face function n . (P - U) at any voxel center P, or at the center one
// voxel past the grid along z (P_z <= 1.5 * 2^16, so |P - U| <= 1.75 * 2^16
// = 2^16.81), is below 3 * 2^34.17 * 2^16.81 = 2^52.56 in magnitude.  Every
// partial sum and product below therefore stays under 2^53 and is exact in
// IEEE double, which gfx950 executes at full rate;
// the double type is used as an exact 53-bit integer carrier, never for a
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
constexpr uint32_t kStatusFull = 4u;   // sparse output: more bricks than the pool holds

struct GridGeom {
    int32_t n[3];      // voxels per axis (powers of two)
    int32_t shift[3];  // log2 of the voxel pitch 2S in lattice units
    int32_t half[3];   // S = 2^15 / n
    int32_t words;     // W = ceil(nz / 32) words per column
};

__device__ __forceinline__ bool index_ok(int32_t x, int64_t nv) {
    return x >= 0 && (int64_t)x < nv;
}

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

// Candidate box of a tet (inclusive voxel index ranges); false when empty.
__device__ __forceinline__ bool candidate_box(const int4 &A, const int4 &B, const int4 &C,
                                              const int4 &D, const GridGeom &g, int32_t lo[3],
                                              int32_t hi[3]) {
    const int32_t mn[3] = {min(min(A.x, B.x), min(C.x, D.x)), min(min(A.y, B.y), min(C.y, D.y)),
                           min(min(A.z, B.z), min(C.z, D.z))};
    const int32_t mx[3] = {max(max(A.x, B.x), max(C.x, D.x)), max(max(A.y, B.y), max(C.y, D.y)),
                           max(max(A.z, B.z), max(C.z, D.z))};
#pragma unroll
    for (int a = 0; a < 3; ++a) axis_range(mn[a], mx[a], g.half[a], g.shift[a], g.n[a], lo[a], hi[a]);
    return lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2];
}

// The half-open tie rule: a face function that is exactly zero at a center
// counts as positive iff its gradient is lexicographically positive in the
// order (z, y, x) -- the sign it takes after the push eps*ez + eps^2*ey +
// eps^3*ex.
__device__ __forceinline__ bool lex_positive(double gx, double gy, double gz) {
    return gz > 0.0 || (gz == 0.0 && (gy > 0.0 || (gy == 0.0 && gx > 0.0)));
}

// One face of a tet in "threshold form", relative to the first candidate
// center (i0, j0, k0) of a box.  For the column (i0+di, j0+dj):
//     a(di, dj) = A + SX*di + SY*dj
// and the face admits dk exactly for dk >= t or dk < t (see lower), where
// t is the smallest integer dk >= 0 with a + S*dk >= 0 (t = ceil(-a/S)).
// Lower faces (gradient z > 0, and vertical faces) give the span's start,
// upper faces its end.  A vertical face (S = 0) stores R = 2^60 so that the
// same formula yields t = 0 (whole column in) for a >= 0 and t = everything
// for a < 0.  All values are exact integers held in doubles, except R.
struct Face {
    double A, SX, SY, S;
    float R;  // estimate of 1/S (relative error < 2^-22), or 2^60 when S = 0
};

// Builds the four faces of tet (A,B,C,D) (lattice coordinates) relative to
// the voxel center p0.  Returns false for a degenerate tet.  lower_mask bit f
// is set when face f bounds the span from below.
//
// The face opposite vertex X through (U,V,W) has normal (V-U) x (W-U),
// flipped so that X lies on its positive side; L(P) = n . (P - U) is
// |6 vol| times X's barycentric coordinate at P -- the affine function whose
// sign Theorem 1's determinant of that face decides.  The center is on the
// inner side iff L + c >= 0, with c = 0 when a zero counts as inside (tie
// rule: n lexicographically positive; never in strict mode) and c = -1
// otherwise.  Along a column L = L0 + sz*dk with sz = n_z * 2Sz:
//   sz > 0 (lower face): admitted dk are those >= the first dk with
//          (L0 + c) + sz*dk >= 0;
//   sz < 0 (upper face): admitted dk are those below the first dk with
//          L0 + c + sz*dk < 0, i.e. with (-L0 - c - 1) + (-sz)*dk >= 0;
//   sz = 0 (vertical face): every dk or none, by the sign of L0 + c.
__device__ __forceinline__ bool build_faces(const int4 &A, const int4 &B, const int4 &C,
                                            const int4 &D, const double p0[3],
                                            const GridGeom &g, bool strict, Face f[4],
                                            uint32_t &lower_mask) {
    const double v[4][3] = {{(double)A.x, (double)A.y, (double)A.z},
                            {(double)B.x, (double)B.y, (double)B.z},
                            {(double)C.x, (double)C.y, (double)C.z},
                            {(double)D.x, (double)D.y, (double)D.z}};
    // (opposite vertex, three face vertices)
    const int tri[4][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {2, 0, 1, 3}, {3, 0, 1, 2}};
    // The side of X relative to face (U,V,W) is det[V-U, W-U, X-U], the
    // orientation of (U,V,W,X): an alternating function of the four points,
    // so every face's side is +-vol with vol = orientation(0,1,2,3), the sign
    // given by the parity of (U,V,W,X) as a permutation of (0,1,2,3): odd
    // for faces 0 and 2, even for faces 1 and 3.  vol is exact (below 2^53).
    const double d1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double d2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double d3[3] = {v[3][0] - v[0][0], v[3][1] - v[0][1], v[3][2] - v[0][2]};
    const double vol = (d1[1] * d2[2] - d1[2] * d2[1]) * d3[0] + (d1[2] * d2[0] - d1[0] * d2[2]) * d3[1] +
                       (d1[0] * d2[1] - d1[1] * d2[0]) * d3[2];
    if (vol == 0.0) return false;
    const double oD = vol < 0.0 ? -1.0 : 1.0;
    lower_mask = 0;
#pragma unroll
    for (int fi = 0; fi < 4; ++fi) {
        const double *U = v[tri[fi][1]], *V = v[tri[fi][2]], *Wv = v[tri[fi][3]];
        const double e1[3] = {V[0] - U[0], V[1] - U[1], V[2] - U[2]};
        const double e2[3] = {Wv[0] - U[0], Wv[1] - U[1], Wv[2] - U[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
        const double o = (fi & 1) ? oD : -oD;
        n[0] *= o;
        n[1] *= o;
        n[2] *= o;
        // inside iff L + c >= 0, c = 0 when a zero counts as inside else -1
        const double c = (!strict && lex_positive(n[0], n[1], n[2])) ? 0.0 : -1.0;
        const double L0 =
            n[0] * (p0[0] - U[0]) + n[1] * (p0[1] - U[1]) + n[2] * (p0[2] - U[2]) + c;
        const double sx = n[0] * (double)(2 * g.half[0]);
        const double sy = n[1] * (double)(2 * g.half[1]);
        const double sz = n[2] * (double)(2 * g.half[2]);
        // lower (or vertical, sz >= 0): span starts at the first dk with
        // L0 + sz dk >= 0.  Upper (sz < 0): span ends at the first dk with
        // L0 + sz dk < 0, i.e. with -(L0 + sz dk) - 1 >= 0.  Both in the form
        // A + S dk >= 0 with S >= 0.
        const bool up = sz < 0.0;
        const double sg = up ? -1.0 : 1.0;
        f[fi].A = fma(sg, L0, up ? -1.0 : 0.0);
        f[fi].SX = sg * sx;
        f[fi].SY = sg * sy;
        f[fi].S = sg * sz;
        f[fi].R = f[fi].S > 0.0 ? __builtin_amdgcn_rcpf((float)f[fi].S)
                                : 1152921504606846976.0f;  // 2^60
        lower_mask |= up ? 0u : 1u << fi;
    }
    return true;
}

// First dk in [0, nk + 1] with a + S*dk >= 0 (at least nk when none in
// [0, nk-1]).  With x = -a/S the threshold is t = ceil(x).  R is the
// hardware single-precision reciprocal of S rounded to float (S >= 1, so no
// denormals): rounding S costs at most 2^-24 and the reciprocal 1 ulp
// (2^-23), so R is within 2^-22 of 1/S relatively (the argument below holds
// up to 2^-21).  The estimate y = fma(-a, R, -1/2) then lies, for |x| <= 2^20,
// in [x - 0.75, x - 0.25], strictly between x - 1 and x, so ceil(y) is t or
// t - 1; for larger |x| (nk <= 2^15) y and x have the same sign and both
// exceed nk in magnitude, so they clamp to the same end of [0, nk].  One
// exact evaluation of a + S*e at e <= nk (a center at most one voxel past
// the box, still inside the exactness bound) fixes the estimate.
__device__ __forceinline__ int32_t face_threshold(const Face &f, double a, double nkd) {
    double e = ceil(fma(-a, (double)f.R, -0.5));
    e = fmin(fmax(e, 0.0), nkd);
    const bool up = fma(f.S, e, a) < 0.0;
    return (int32_t)e + (up ? 1 : 0);
}

// ORs the bit run [k_lo, k_hi) (k_lo < k_hi, word-relative indices) into a
// word array with device-scope atomics.
__device__ __forceinline__ void or_run_global(uint32_t *col, int32_t k_lo, int32_t k_hi) {
    const int32_t w0 = k_lo >> 5, w1 = (k_hi - 1) >> 5;
    for (int32_t w = w0; w <= w1; ++w) {
        uint32_t m = 0xffffffffu;
        if (w == w0) m &= 0xffffffffu << (k_lo & 31);
        if (w == w1) m &= 0xffffffffu >> (31 - ((k_hi - 1) & 31));
        __hip_atomic_fetch_or(col + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Same for a word array in LDS, written for the common run inside one
// word: the first word unconditionally, whole words between, the last word
// when it is another.
__device__ __forceinline__ void or_run_lds(uint32_t *col, int32_t k_lo, int32_t k_hi) {
    const int32_t w0 = k_lo >> 5, w1 = (k_hi - 1) >> 5;
    const uint32_t mlo = 0xffffffffu << (k_lo & 31);
    const uint32_t mhi = 0xffffffffu >> (31 - ((k_hi - 1) & 31));
    atomicOr(col + w0, w0 == w1 ? mlo & mhi : mlo);
    if (w1 > w0) {
        for (int32_t w = w0 + 1; w < w1; ++w) atomicOr(col + w, 0xffffffffu);
        atomicOr(col + w1, mhi);
    }
}

}  // namespace tv
