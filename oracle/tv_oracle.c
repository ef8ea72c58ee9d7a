/*
 * tv_oracle.c -- plain, slow, obviously correct CPU voxelizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or constant generator with the
 * HIP library.
 *
 * What it computes (the paper's voxelization, Section 3 "Voxelization" and
 * Section 4, Theorem 1):
 *   for every tetrahedron, scan the voxel centers inside its axis-aligned
 *   bounding box and set the voxel when the center lies inside the tet, with
 *   the inside test of Theorem 1: with a = A-P, b = B-P, c = C-P, d = D-P and
 *     Da = det[b;c;d], Db = det[a;c;d], Dc = det[a;b;d], Dd = det[a;b;c]
 *   (rows are the vectors), P is inside iff
 *     (Da>0, Db<0, Dc>0, Dd<0)  or  (Da<0, Db>0, Dc<0, Dd>0).
 *
 * Readings where the paper is silent:
 *   - the sample point of voxel (i,j,k) is its center;
 *   - coordinates live on a fixed-point lattice of 2^16 units per bbox extent
 *     and the center of voxel (i,j,k) is ((2i+1)Sx, (2j+1)Sy, (2k+1)Sz) with
 *     S = 2^15 / N per axis (N a power of two);
 *   - TIE RULE (mode ORACLE_HALF_OPEN): a determinant that is exactly zero at
 *     P takes the sign it has at P + eps*ez + eps^2*ey + eps^3*ex for
 *     infinitesimal eps > 0.  Each determinant is an affine function of P,
 *     so that sign is the sign of the first non-zero of the finite
 *     differences D(P+ez)-D(P), D(P+ey)-D(P), D(P+ex)-D(P).  Mode
 *     ORACLE_STRICT applies Theorem 1 literally (a zero never matches);
 *   - degenerate tets (zero signed volume, Lemma 1.1's det/6) add nothing;
 *   - overlapping tets give the union of their voxels.
 *
 * The snap (fp32 world coordinate -> lattice) follows the library contract:
 *   q = rint(((double)v - (double)lo) * 65536.0 / ((double)hi - (double)lo))
 * evaluated left to right in IEEE double with round-to-nearest-even and no
 * fused multiply-add; a NaN or a q outside [-2^14, 2^16 + 2^14] is an error.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_DIMS (-2)
#define ORACLE_ERR_INDEX (-3)
#define ORACLE_ERR_RANGE (-4)
#define ORACLE_ERR_NOMEM (-6)

#define ORACLE_HALF_OPEN 0
#define ORACLE_STRICT 1

#define LATTICE 65536
#define Q_LO (-16384)
#define Q_HI (65536 + 16384)

/* ------------------------------------------------------------------ snap */

int oracle_snap(const float *v, int64_t nv, const float *lo, const float *hi, int32_t *q)
{
    for (int a = 0; a < 3; ++a) {
        if (!(hi[a] > lo[a])) return ORACLE_ERR_ARG;
    }
    for (int64_t i = 0; i < nv; ++i) {
        for (int a = 0; a < 3; ++a) {
            double t = (double)v[3 * i + a] - (double)lo[a];
            t = t * 65536.0;
            t = t / ((double)hi[a] - (double)lo[a]);
            if (isnan(t)) return ORACLE_ERR_RANGE;
            double r = nearbyint(t); /* default rounding mode: ties to even */
            if (r < (double)Q_LO || r > (double)Q_HI) return ORACLE_ERR_RANGE;
            q[3 * i + a] = (int32_t)r;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------- determinants */

/* det of the 3x3 matrix whose rows are r0, r1, r2 */
static int64_t det3(const int64_t r0[3], const int64_t r1[3], const int64_t r2[3])
{
    return r0[0] * (r1[1] * r2[2] - r1[2] * r2[1])
         - r0[1] * (r1[0] * r2[2] - r1[2] * r2[0])
         + r0[2] * (r1[0] * r2[1] - r1[1] * r2[0]);
}

/* The four determinants of Theorem 1 at point P, in the order Da, Db, Dc, Dd. */
static void theorem1_dets(const int64_t P[3], const int64_t A[3], const int64_t B[3],
                          const int64_t C[3], const int64_t D[3], int64_t out[4])
{
    int64_t a[3], b[3], c[3], d[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = A[k] - P[k];
        b[k] = B[k] - P[k];
        c[k] = C[k] - P[k];
        d[k] = D[k] - P[k];
    }
    out[0] = det3(b, c, d);
    out[1] = det3(a, c, d);
    out[2] = det3(a, b, d);
    out[3] = det3(a, b, c);
}

static int sgn64(int64_t x) { return (x > 0) - (x < 0); }

/* Signs of Da..Dd at P; in half-open mode a zero takes the sign at the
 * perturbed point P + eps*ez + eps^2*ey + eps^3*ex (eps -> 0+). */
static void theorem1_signs(const int64_t P[3], const int64_t A[3], const int64_t B[3],
                           const int64_t C[3], const int64_t D[3], int mode, int s[4])
{
    int64_t d0[4];
    theorem1_dets(P, A, B, C, D, d0);
    int any_zero = 0;
    for (int f = 0; f < 4; ++f) {
        s[f] = sgn64(d0[f]);
        any_zero |= (s[f] == 0);
    }
    if (!any_zero || mode == ORACLE_STRICT) return;
    /* perturbation order: z first, then y, then x */
    static const int axis_order[3] = {2, 1, 0};
    for (int step = 0; step < 3; ++step) {
        int64_t Pn[3] = {P[0], P[1], P[2]};
        Pn[axis_order[step]] += 1;
        int64_t d1[4];
        theorem1_dets(Pn, A, B, C, D, d1);
        int still_zero = 0;
        for (int f = 0; f < 4; ++f) {
            if (s[f] == 0) {
                /* the determinant is affine in P: d1 - d0 is its exact partial
                 * derivative along this axis */
                s[f] = sgn64(d1[f] - d0[f]);
                /* a zero derivative leaves the sign undecided for the next axis */
                still_zero |= (s[f] == 0);
            }
        }
        if (!still_zero) return;
        /* the undecided ones are re-tested against the original point on the
         * next axis (d0 is unchanged) */
    }
}

static int theorem1_inside(const int s[4])
{
    return (s[0] > 0 && s[1] < 0 && s[2] > 0 && s[3] < 0) ||
           (s[0] < 0 && s[1] > 0 && s[2] < 0 && s[3] > 0);
}

/* Six times the signed volume (Lemma 1.1): det of the rows AB, AC, AD. */
static int64_t six_volume(const int64_t A[3], const int64_t B[3], const int64_t C[3],
                          const int64_t D[3])
{
    int64_t ab[3], ac[3], ad[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = B[k] - A[k];
        ac[k] = C[k] - A[k];
        ad[k] = D[k] - A[k];
    }
    return det3(ab, ac, ad);
}

/* Exported single-point predicate: 1 if P is inside tet ABCD under `mode`. */
int oracle_point_in_tet(const int64_t *P, const int64_t *A, const int64_t *B,
                        const int64_t *C, const int64_t *D, int mode)
{
    if (six_volume(A, B, C, D) == 0) return 0;
    int s[4];
    theorem1_signs(P, A, B, C, D, mode, s);
    return theorem1_inside(s);
}

/* Exported: the four raw determinants (for identity checks in the tests). */
void oracle_theorem1_dets(const int64_t *P, const int64_t *A, const int64_t *B,
                          const int64_t *C, const int64_t *D, int64_t *out)
{
    theorem1_dets(P, A, B, C, D, out);
}

int64_t oracle_six_volume(const int64_t *A, const int64_t *B, const int64_t *C,
                          const int64_t *D)
{
    return six_volume(A, B, C, D);
}

/* ------------------------------------------------------------ voxelize */

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static int64_t ceil_div(int64_t a, int64_t b) /* b > 0 */
{
    return -floor_div(-a, b);
}

static int is_pow2_dim(int n) { return n >= 1 && n <= 32768 && (n & (n - 1)) == 0; }

typedef struct {
    const int32_t *q;
    int64_t nv;
    const int32_t *tets;
    int64_t t0, t1;
    int n[3];
    int64_t win_lo[3], win_hi[3]; /* inclusive voxel-index window */
    int mode;
    int brute; /* 1: test every center of the window against every tet */
    uint32_t *words;
    uint8_t *cover; /* optional saturating per-voxel coverage count */
    int status;
} job_t;

static void *voxelize_range(void *arg)
{
    job_t *J = (job_t *)arg;
    const int64_t W = (J->n[2] + 31) / 32;
    int64_t S[3];
    for (int a = 0; a < 3; ++a) S[a] = (LATTICE / 2) / J->n[a];
    for (int64_t t = J->t0; t < J->t1; ++t) {
        int64_t V[4][3];
        for (int v = 0; v < 4; ++v) {
            int32_t id = J->tets[4 * t + v];
            if (id < 0 || id >= J->nv) {
                J->status = ORACLE_ERR_INDEX;
                return NULL;
            }
            for (int a = 0; a < 3; ++a) V[v][a] = J->q[3 * (int64_t)id + a];
        }
        if (six_volume(V[0], V[1], V[2], V[3]) == 0) continue;
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            if (J->brute) {
                lo[a] = J->win_lo[a];
                hi[a] = J->win_hi[a];
                continue;
            }
            int64_t mn = V[0][a], mx = V[0][a];
            for (int v = 1; v < 4; ++v) {
                if (V[v][a] < mn) mn = V[v][a];
                if (V[v][a] > mx) mx = V[v][a];
            }
            /* centers (2i+1)S with mn <= (2i+1)S <= mx */
            lo[a] = ceil_div(mn - S[a], 2 * S[a]);
            hi[a] = floor_div(mx - S[a], 2 * S[a]);
            if (lo[a] < J->win_lo[a]) lo[a] = J->win_lo[a];
            if (hi[a] > J->win_hi[a]) hi[a] = J->win_hi[a];
        }
        for (int64_t i = lo[0]; i <= hi[0]; ++i)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t k = lo[2]; k <= hi[2]; ++k) {
                    int64_t P[3] = {(2 * i + 1) * S[0], (2 * j + 1) * S[1], (2 * k + 1) * S[2]};
                    int s[4];
                    theorem1_signs(P, V[0], V[1], V[2], V[3], J->mode, s);
                    if (!theorem1_inside(s)) continue;
                    int64_t col = i * J->n[1] + j;
                    J->words[col * W + (k >> 5)] |= (uint32_t)1u << (k & 31);
                    if (J->cover) {
                        uint8_t *c = &J->cover[(col * J->n[2]) + k];
                        if (*c < 255) *c += 1;
                    }
                }
    }
    return NULL;
}

/*
 * Voxelize lattice vertices q[nv][3] and tets[nt][4] into words (zeroed here;
 * nx*ny*ceil(nz/32) uint32, voxel (i,j,k) is bit k%32 of word
 * (i*ny + j)*W + k/32).  Only voxels inside the inclusive index window
 * win[0..5] = {i0,i1,j0,j1,k0,k1} are set (pass NULL for the whole grid).
 * cover (optional, nx*ny*nz bytes, zeroed here) counts covering tets;
 * requesting it forces one thread.  brute != 0 tests every window center
 * against every tet (no bounding-box culling).
 */
int oracle_voxelize(const int32_t *q, int64_t nv, const int32_t *tets, int64_t nt, int nx,
                    int ny, int nz, const int64_t *win, int mode, int brute, int nthreads,
                    uint32_t *words, uint8_t *cover)
{
    if (!is_pow2_dim(nx) || !is_pow2_dim(ny) || !is_pow2_dim(nz)) return ORACLE_ERR_DIMS;
    if (nv < 0 || nt < 0 || (nt > 0 && (!q || !tets)) || !words) return ORACLE_ERR_ARG;
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (q[i] < Q_LO || q[i] > Q_HI) return ORACLE_ERR_RANGE;
    const int64_t W = (nz + 31) / 32;
    const int64_t nwords = (int64_t)nx * ny * W;
    memset(words, 0, (size_t)nwords * 4);
    if (cover) {
        memset(cover, 0, (size_t)nx * ny * nz);
        nthreads = 1;
    }
    int64_t wl[3] = {0, 0, 0}, wh[3] = {nx - 1, ny - 1, nz - 1};
    if (win) {
        for (int a = 0; a < 3; ++a) {
            wl[a] = win[2 * a] < 0 ? 0 : win[2 * a];
            wh[a] = win[2 * a + 1] > wh[a] ? wh[a] : win[2 * a + 1];
        }
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nt < 4096) nthreads = 1;
    job_t jobs[256];
    pthread_t th[256];
    uint32_t *priv[256];
    int n3[3] = {nx, ny, nz};
    for (int t = 0; t < nthreads; ++t) {
        job_t *J = &jobs[t];
        J->q = q;
        J->nv = nv;
        J->tets = tets;
        J->t0 = nt * t / nthreads;
        J->t1 = nt * (t + 1) / nthreads;
        memcpy(J->n, n3, sizeof n3);
        memcpy(J->win_lo, wl, sizeof wl);
        memcpy(J->win_hi, wh, sizeof wh);
        J->mode = mode;
        J->brute = brute;
        J->cover = cover;
        J->status = ORACLE_OK;
        if (t == 0) {
            priv[t] = words;
        } else {
            priv[t] = (uint32_t *)calloc((size_t)nwords, 4);
            if (!priv[t]) {
                for (int u = 1; u < t; ++u) free(priv[u]);
                return ORACLE_ERR_NOMEM;
            }
        }
        J->words = priv[t];
    }
    if (nthreads == 1) {
        voxelize_range(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, voxelize_range, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    int status = ORACLE_OK;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status != ORACLE_OK) status = jobs[t].status;
        if (t > 0) {
            for (int64_t w = 0; w < nwords; ++w) words[w] |= priv[t][w];
            free(priv[t]);
        }
    }
    return status;
}
