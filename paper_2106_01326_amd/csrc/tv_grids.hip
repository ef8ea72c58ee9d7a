// Consumers of a voxel grid on the device: dense tensors for 3D CNNs
// (the paper's motivating use, Section 1, left as future work in
// Section 6), coarser occupancy levels, and sparse bricks (the sparse-storage
// concern of the Octrees paragraph of Section 5).  All three read the
// packed layout of include/tv.h and are bound by HBM traffic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "tv.h"
#include "tv_internal.h"

namespace {

bool pow2_dim(int32_t n) { return n >= 1 && n <= 32768 && (n & (n - 1)) == 0; }

bool dims_ok(tv_dims d) { return pow2_dim(d.nx) && pow2_dim(d.ny) && pow2_dim(d.nz); }

tv_status launched(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tv::set_error(TV_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return TV_OK;
}

constexpr int kThreads = 256;

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// ---------------------------------------------------------------- unpack

// One thread per V consecutive outputs (16 bytes: V = 16 bytes or 4 floats)
// along z; nz is a multiple of V, so a thread's outputs share one column and
// one word.  Consecutive threads write consecutive 16-byte pieces.
template <int V>
__global__ void __launch_bounds__(kThreads)
    k_unpack16(const uint32_t *__restrict__ grid, int32_t nz, int32_t words, int64_t nchunks,
               uint4 *__restrict__ out) {
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= nchunks) return;
    const int64_t first = o * V;  // first output voxel (column-major, z fastest)
    const int64_t col = first / nz;
    const int32_t k = (int32_t)(first - col * nz);
    const uint32_t bits = grid[col * words + (k >> 5)] >> (k & 31);
    uint4 r;
    if (V == 16) {
        // 16 bytes, each 0 or 1: nibble q of `bits` becomes the four bytes of word q
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t x = (bits >> (4 * q)) & 15u;
            w[q] = (x & 1u) | ((x & 2u) << 7) | ((x & 4u) << 14) | ((x & 8u) << 21);
        }
        r = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        const uint32_t one = 0x3f800000u;  // 1.0f
        r = make_uint4((bits & 1u) ? one : 0u, (bits & 2u) ? one : 0u, (bits & 4u) ? one : 0u,
                       (bits & 8u) ? one : 0u);
    }
    out[o] = r;
}

// Any nz: one thread per output voxel.
template <typename T>
__global__ void __launch_bounds__(kThreads)
    k_unpack1(const uint32_t *__restrict__ grid, int32_t nz, int32_t words, int64_t n,
              T *__restrict__ out) {
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= n) return;
    const int64_t col = o / nz;
    const int32_t k = (int32_t)(o - col * nz);
    out[o] = (T)((grid[col * words + (k >> 5)] >> (k & 31)) & 1u);
}

// ------------------------------------------------------------------ pool

// Fraction pooling by f (f divides 32 and every dim): one thread per
// (I, J, input word) computes the 32/f (or nz/f) outputs of that z range
// from the f*f words of its columns.
__global__ void __launch_bounds__(kThreads)
    k_pool_fraction(const uint32_t *__restrict__ grid, int32_t ny, int32_t nz, int32_t words,
                    int32_t f, int32_t lf, int64_t nthreads, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= nthreads) return;
    const int32_t nyo = ny >> lf, nzo = nz >> lf;
    const int32_t wi = (int32_t)(t % words);
    const int64_t ij = t / words;
    const int32_t J = (int32_t)(ij % nyo), I = (int32_t)(ij / nyo);
    const int32_t per = min(32, nz) >> lf;  // outputs from this word
    uint32_t cnt[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) cnt[q] = 0;
    const uint32_t mask = f == 32 ? 0xffffffffu : ((1u << f) - 1u);
    for (int32_t di = 0; di < f; ++di)
        for (int32_t dj = 0; dj < f; ++dj) {
            const int64_t col = (int64_t)((I << lf) + di) * ny + ((J << lf) + dj);
            const uint32_t w = grid[col * words + wi];
#pragma unroll
            for (int q = 0; q < 32; ++q)
                if (q < per) cnt[q] += (uint32_t)__popc((w >> (q << lf)) & mask);
        }
    const float scale = 1.0f / (float)(f * f * f);
    float *o = out + ((int64_t)I * nyo + J) * nzo + (int64_t)wi * (32 >> lf);
#pragma unroll
    for (int q = 0; q < 32; ++q)
        if (q < per) o[q] = (float)cnt[q] * scale;
}

// Fraction pooling for f <= 8 with nz/f a multiple of 4: one thread per 4
// consecutive outputs along z (one float4), so consecutive threads write
// consecutive 16-byte pieces; their 4f input bits lie in one word.
__global__ void __launch_bounds__(kThreads)
    k_pool_fraction4(const uint32_t *__restrict__ grid, int32_t ny, int32_t nz, int32_t words,
                     int32_t f, int32_t lf, int64_t nthreads, float4 *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= nthreads) return;
    const int32_t nyo = ny >> lf, nzo4 = (nz >> lf) >> 2;
    const int32_t k4 = (int32_t)(t % nzo4);
    const int64_t ij = t / nzo4;
    const int32_t J = (int32_t)(ij % nyo), I = (int32_t)(ij / nyo);
    const int32_t z0 = (k4 << 2) << lf;  // first input z
    const int32_t wi = z0 >> 5, sh = z0 & 31;
    const uint32_t mask = (1u << f) - 1u;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int32_t di = 0; di < f; ++di)
        for (int32_t dj = 0; dj < f; ++dj) {
            const int64_t col = (int64_t)((I << lf) + di) * ny + ((J << lf) + dj);
            const uint32_t w = grid[col * words + wi] >> sh;
            c0 += (uint32_t)__popc(w & mask);
            c1 += (uint32_t)__popc((w >> f) & mask);
            c2 += (uint32_t)__popc((w >> (2 * f)) & mask);
            c3 += (uint32_t)__popc((w >> (3 * f)) & mask);
        }
    const float scale = 1.0f / (float)(f * f * f);
    out[t] = make_float4((float)c0 * scale, (float)c1 * scale, (float)c2 * scale, (float)c3 * scale);
}

// Any-pooling by f into a packed grid of dims / f: one thread per output
// word, reading the f * f columns and the f input words per column that
// cover its 32 (or fewer) output voxels.
__global__ void __launch_bounds__(kThreads)
    k_pool_any(const uint32_t *__restrict__ grid, int32_t ny, int32_t nz, int32_t words,
               int32_t f, int32_t lf, int32_t words_out, int64_t nthreads,
               uint32_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= nthreads) return;
    const int32_t nyo = ny >> lf, nzo = nz >> lf;
    const int32_t wo = (int32_t)(t % words_out);
    const int64_t ij = t / words_out;
    const int32_t J = (int32_t)(ij % nyo), I = (int32_t)(ij / nyo);
    const int32_t kout = min(32, nzo - 32 * wo);     // output voxels in this word
    const int32_t kin = kout << lf;                 // input z voxels they cover
    const int32_t w0 = wo << lf;                    // first input word
    const int32_t nw = (kin + 31) >> 5;             // input words per column
    const int32_t per = min(32, kin) >> lf;         // outputs per input word
    uint32_t acc = 0;
    for (int32_t di = 0; di < f; ++di)
        for (int32_t dj = 0; dj < f; ++dj) {
            const int64_t col = (int64_t)((I << lf) + di) * ny + ((J << lf) + dj);
            for (int32_t q = 0; q < nw; ++q) {
                const uint32_t w = grid[col * words + w0 + q];
                if (w == 0u) continue;
                const uint32_t mask = f == 32 ? 0xffffffffu : ((1u << f) - 1u);
                for (int32_t g = 0; g < per; ++g)
                    if ((w >> (g << lf)) & mask) acc |= 1u << (q * per + g);
            }
        }
    out[ij * words_out + wo] = acc;
}

// ---------------------------------------------------------------- bricks

// A brick is 8 x 8 columns by 32 z (one word per column, 256 bytes); brick
// (bx, by, bz) has id (bx * nby + by) * nbz + bz and holds the words of
// columns (8bx + u, 8by + v), u, v < 8, word bz, in u-major order.
constexpr int kBrickCols = 8;

__device__ __forceinline__ bool brick_nonzero(const uint32_t *__restrict__ grid, int32_t ny,
                                              int32_t words, int32_t nby, int32_t nbz,
                                              int64_t id) {
    const int32_t bz = (int32_t)(id % nbz);
    const int64_t bxy = id / nbz;
    const int32_t by = (int32_t)(bxy % nby), bx = (int32_t)(bxy / nby);
    uint32_t any = 0;
    for (int u = 0; u < kBrickCols; ++u)
        for (int v = 0; v < kBrickCols; ++v)
            any |= grid[((int64_t)(kBrickCols * bx + u) * ny + kBrickCols * by + v) * words + bz];
    return any != 0u;
}

// Pass 1: non-empty bricks per block of kThreads brick ids.
__global__ void __launch_bounds__(kThreads)
    k_brick_count(const uint32_t *__restrict__ grid, int32_t ny, int32_t words, int32_t nby,
                  int32_t nbz, int64_t nbricks, uint32_t *__restrict__ block_count) {
    const int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool nz = id < nbricks && brick_nonzero(grid, ny, words, nby, nbz, id);
    const uint64_t b = __ballot(nz);
    __shared__ uint32_t s_w[kThreads / 64];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += s_w[w];
        block_count[blockIdx.x] = s;
    }
}

// Pass 2: exclusive scan of the block counts in place (one workgroup);
// total[0] = number of non-empty bricks.
__global__ void __launch_bounds__(1024)
    k_brick_scan(uint32_t *__restrict__ block_count, int64_t nblocks, uint32_t *__restrict__ total) {
    __shared__ uint32_t s[1024];
    __shared__ uint32_t s_base;
    const int tid = threadIdx.x;
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblocks; base += 1024) {
        const int64_t i = base + tid;
        const uint32_t c = i < nblocks ? block_count[i] : 0u;
        s[tid] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t a = tid >= off ? s[tid - off] : 0u;
            __syncthreads();
            s[tid] += a;
            __syncthreads();
        }
        if (i < nblocks) block_count[i] = s_base + s[tid] - c;
        __syncthreads();
        if (tid == 1023) s_base += s[1023];
        __syncthreads();
    }
    if (tid == 0) total[0] = s_base;
}

// Pass 3: every non-empty brick takes slot (block offset + rank in block);
// slots below `capacity` receive the id and the 64 words.
__global__ void __launch_bounds__(kThreads)
    k_brick_write(const uint32_t *__restrict__ grid, int32_t ny, int32_t words, int32_t nby,
                  int32_t nbz, int64_t nbricks, const uint32_t *__restrict__ block_off,
                  int64_t capacity, uint32_t *__restrict__ ids, uint32_t *__restrict__ bwords) {
    const int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool nz = id < nbricks && brick_nonzero(grid, ny, words, nby, nbz, id);
    const uint64_t b = __ballot(nz);
    __shared__ uint32_t s_w[kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) s_w[wv] = (uint32_t)__popcll(b);
    __syncthreads();
    if (!nz) return;
    uint32_t rank = (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) rank += s_w[w];
    const int64_t slot = (int64_t)block_off[blockIdx.x] + rank;
    if (slot >= capacity) return;
    ids[slot] = (uint32_t)id;
    const int32_t bz = (int32_t)(id % nbz);
    const int64_t bxy = id / nbz;
    const int32_t by = (int32_t)(bxy % nby), bx = (int32_t)(bxy / nby);
    uint4 *dst = reinterpret_cast<uint4 *>(bwords + slot * (kBrickCols * kBrickCols));
    for (int u = 0; u < kBrickCols; ++u) {
        const int64_t c0 = (int64_t)(kBrickCols * bx + u) * ny + kBrickCols * by;
        uint32_t w[kBrickCols];
#pragma unroll
        for (int v = 0; v < kBrickCols; ++v) w[v] = grid[(c0 + v) * words + bz];
        dst[2 * u] = make_uint4(w[0], w[1], w[2], w[3]);
        dst[2 * u + 1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
}

// ----------------------------------------------------------- batch export

// One grid of a batch export: device pointer, log2 of its dims, words per
// column.
struct ExportRef {
    const uint32_t *grid;
    int32_t ln[3];
    int32_t words;
};

// Set voxels of the source block of output cell c of grid g (per axis a
// block of 2^(ln - lres) voxels on a pooled axis, the one voxel it repeats
// otherwise), counted word by word along z; lblock = log2 of the block size.
__device__ __forceinline__ uint32_t export_count(const ExportRef &g, const int32_t c[3], int32_t lres,
                                                 int32_t &lblock) {
    int32_t lo[3], len[3];
    lblock = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t d = g.ln[a] - lres;
        lo[a] = d >= 0 ? c[a] << d : c[a] >> -d;
        len[a] = d >= 0 ? 1 << d : 1;
        lblock += d >= 0 ? d : 0;
    }
    const int32_t k0 = lo[2], k1 = lo[2] + len[2] - 1, w0 = k0 >> 5, w1 = k1 >> 5;
    uint32_t cnt = 0;
    for (int32_t i = lo[0]; i < lo[0] + len[0]; ++i)
        for (int32_t j = lo[1]; j < lo[1] + len[1]; ++j) {
            const uint32_t *col = g.grid + (((int64_t)i << g.ln[1]) + j) * g.words;
            for (int32_t w = w0; w <= w1; ++w) {
                uint32_t m = 0xffffffffu;
                if (w == w0) m &= 0xffffffffu << (k0 & 31);
                if (w == w1) m &= 0xffffffffu >> (31 - (k1 & 31));
                cnt += (uint32_t)__popc(col[w] & m);
            }
        }
    return cnt;
}

// One thread per V consecutive output cells along z (grid-stride; V = 4
// when res is a multiple of 4, so a thread writes one float4 or 4 bytes).
// A block holds at most 2^24 voxels, so the count and the fraction
// (count * 2^-lblock) are exact in float.
template <bool kFraction, int V>
__global__ void __launch_bounds__(kThreads)
    k_export(const ExportRef *__restrict__ tab, int64_t total, int32_t lres, void *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int32_t cmask = (1 << lres) - 1;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total / V; t += stride) {
        const int64_t o = t * V;
        const ExportRef g = tab[o >> (3 * lres)];
        int32_t c[3] = {(int32_t)(o >> (2 * lres)) & cmask, (int32_t)(o >> lres) & cmask, (int32_t)o & cmask};
        float f[V];
        uint32_t any = 0;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            int32_t lblock;
            const uint32_t cnt = export_count(g, c, lres, lblock);
            f[q] = ldexpf((float)cnt, -lblock);
            any |= (cnt ? 1u : 0u) << (8 * q);
            ++c[2];
        }
        if (V == 4) {
            if (kFraction) reinterpret_cast<float4 *>(out)[t] = make_float4(f[0], f[1], f[2], f[3]);
            else reinterpret_cast<uint32_t *>(out)[t] = any;
        } else {
            if (kFraction) static_cast<float *>(out)[o] = f[0];
            else static_cast<uint8_t *>(out)[o] = (uint8_t)any;
        }
    }
}

int32_t log2_exact(int32_t n) {
    int32_t l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

extern "C" {

tv_status tv_unpack(const uint32_t *grid, tv_dims dims, void *out, uint32_t format, void *stream) {
    if (!dims_ok(dims))
        return tv::set_error(TV_ERR_UNSUPPORTED_DIMS, "dims (%d, %d, %d)", dims.nx, dims.ny, dims.nz);
    if (!grid || !out) return tv::set_error(TV_ERR_INVALID_ARG, "null grid or output");
    if (format != TV_UNPACK_U8 && format != TV_UNPACK_F32)
        return tv::set_error(TV_ERR_INVALID_ARG, "unknown unpack format %u", format);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t words = (dims.nz + 31) / 32;
    const int64_t n = (int64_t)dims.nx * dims.ny * dims.nz;
    const bool aligned = (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
    if (format == TV_UNPACK_U8) {
        if (dims.nz % 16 == 0 && aligned) {
            const int64_t nch = n / 16;
            k_unpack16<16><<<blocks_for(nch), kThreads, 0, s>>>(grid, dims.nz, words, nch,
                                                                 static_cast<uint4 *>(out));
        } else {
            k_unpack1<uint8_t><<<blocks_for(n), kThreads, 0, s>>>(grid, dims.nz, words, n,
                                                                  static_cast<uint8_t *>(out));
        }
    } else {
        if (dims.nz % 4 == 0 && aligned) {
            const int64_t nch = n / 4;
            k_unpack16<4><<<blocks_for(nch), kThreads, 0, s>>>(grid, dims.nz, words, nch,
                                                                static_cast<uint4 *>(out));
        } else {
            k_unpack1<float><<<blocks_for(n), kThreads, 0, s>>>(grid, dims.nz, words, n,
                                                                static_cast<float *>(out));
        }
    }
    return launched("unpack launch");
}

tv_status tv_pool(const uint32_t *grid, tv_dims dims, int32_t factor, uint32_t mode, void *out,
                  void *stream) {
    if (!dims_ok(dims))
        return tv::set_error(TV_ERR_UNSUPPORTED_DIMS, "dims (%d, %d, %d)", dims.nx, dims.ny, dims.nz);
    if (!grid || !out) return tv::set_error(TV_ERR_INVALID_ARG, "null grid or output");
    if (factor < 2 || factor > 32 || (factor & (factor - 1)) || dims.nx % factor ||
        dims.ny % factor || dims.nz % factor)
        return tv::set_error(TV_ERR_INVALID_ARG,
                             "pool factor %d must be a power of two in [2, 32] dividing every dim",
                             factor);
    if (mode != TV_POOL_FRACTION && mode != TV_POOL_ANY)
        return tv::set_error(TV_ERR_INVALID_ARG, "unknown pool mode %u", mode);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t lf = 0;
    while ((1 << lf) < factor) ++lf;
    const int32_t words = (dims.nz + 31) / 32;
    const int64_t cols_out = (int64_t)(dims.nx / factor) * (dims.ny / factor);
    const bool vec = factor <= 8 && ((dims.nz / factor) & 3) == 0 &&
                     (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
    if (mode == TV_POOL_FRACTION && vec) {
        const int64_t nth = cols_out * (dims.nz / factor / 4);
        k_pool_fraction4<<<blocks_for(nth), kThreads, 0, s>>>(grid, dims.ny, dims.nz, words, factor, lf,
                                                              nth, static_cast<float4 *>(out));
    } else if (mode == TV_POOL_FRACTION) {
        const int64_t nth = cols_out * words;
        k_pool_fraction<<<blocks_for(nth), kThreads, 0, s>>>(grid, dims.ny, dims.nz, words, factor, lf,
                                                             nth, static_cast<float *>(out));
    } else {
        const int32_t words_out = (dims.nz / factor + 31) / 32;
        const int64_t nth = cols_out * words_out;
        k_pool_any<<<blocks_for(nth), kThreads, 0, s>>>(grid, dims.ny, dims.nz, words, factor, lf,
                                                        words_out, nth, static_cast<uint32_t *>(out));
    }
    return launched("pool launch");
}

int64_t tv_brick_count_max(tv_dims dims) {
    if (!dims_ok(dims) || dims.nx % 8 || dims.ny % 8 || dims.nz % 32) return 0;
    return (int64_t)(dims.nx / 8) * (dims.ny / 8) * (dims.nz / 32);
}

size_t tv_bricks_workspace_bytes(tv_dims dims) {
    const int64_t nb = tv_brick_count_max(dims);
    return nb ? (size_t)4 * (size_t)((nb + kThreads - 1) / kThreads) : 0;
}

tv_status tv_bricks(const uint32_t *grid, tv_dims dims, uint32_t *ids, uint32_t *brick_words,
                    int64_t capacity, uint32_t *count, void *ws, size_t ws_bytes, void *stream) {
    const int64_t nb = tv_brick_count_max(dims);
    if (nb == 0)
        return tv::set_error(TV_ERR_UNSUPPORTED_DIMS,
                             "bricks need power-of-two dims with nx, ny multiples of 8 and nz of 32");
    if (!grid || !count || !ws || (capacity > 0 && (!ids || !brick_words)) || capacity < 0)
        return tv::set_error(TV_ERR_INVALID_ARG, "null pointer or negative capacity");
    if ((reinterpret_cast<uintptr_t>(brick_words) & 15u) != 0)
        return tv::set_error(TV_ERR_INVALID_ARG, "brick_words must be 16-byte aligned");
    if (ws_bytes < tv_bricks_workspace_bytes(dims))
        return tv::set_error(TV_ERR_WORKSPACE, "bricks workspace %zu < %zu bytes", ws_bytes,
                             tv_bricks_workspace_bytes(dims));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t words = dims.nz / 32, nby = dims.ny / 8, nbz = dims.nz / 32;
    const int64_t nblocks = (nb + kThreads - 1) / kThreads;
    uint32_t *block = static_cast<uint32_t *>(ws);
    k_brick_count<<<(unsigned)nblocks, kThreads, 0, s>>>(grid, dims.ny, words, nby, nbz, nb, block);
    k_brick_scan<<<1, 1024, 0, s>>>(block, nblocks, count);
    k_brick_write<<<(unsigned)nblocks, kThreads, 0, s>>>(grid, dims.ny, words, nby, nbz, nb, block,
                                                         capacity, ids, brick_words);
    return launched("bricks launch");
}

size_t tv_export_workspace_bytes(int32_t n) {
    if (n <= 0) return 0;
    return ((size_t)n * sizeof(ExportRef) + 255) & ~(size_t)255;
}

tv_status tv_export_batch(const tv_grid_ref *grids, int32_t n, int32_t res, uint32_t mode, void *out,
                          void *ws, size_t ws_bytes, void *stream) {
    if (!grids || n <= 0 || !out)
        return tv::set_error(TV_ERR_INVALID_ARG, "export: need grids, n > 0 and an output");
    if (res < 1 || res > 1024 || (res & (res - 1)))
        return tv::set_error(TV_ERR_INVALID_ARG, "export: res %d is not a power of two in [1, 1024]", res);
    if (mode != TV_EXPORT_FRACTION && mode != TV_EXPORT_ANY)
        return tv::set_error(TV_ERR_INVALID_ARG, "export: unknown mode %u", mode);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < tv_export_workspace_bytes(n))
        return tv::set_error(TV_ERR_WORKSPACE, "export: workspace null, misaligned or below %zu bytes",
                             tv_export_workspace_bytes(n));
    const int32_t lres = log2_exact(res);
    std::vector<ExportRef> tab((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const tv_grid_ref &r = grids[i];
        if (!r.grid) return tv::set_error(TV_ERR_INVALID_ARG, "export: grid %d is null", i);
        if (!dims_ok(r.dims))
            return tv::set_error(TV_ERR_UNSUPPORTED_DIMS, "export: grid %d dims (%d,%d,%d)", i, r.dims.nx,
                                 r.dims.ny, r.dims.nz);
        const int32_t ln[3] = {log2_exact(r.dims.nx), log2_exact(r.dims.ny), log2_exact(r.dims.nz)};
        int32_t lblock = 0;
        for (int a = 0; a < 3; ++a) lblock += ln[a] > lres ? ln[a] - lres : 0;
        if (lblock > 24)
            return tv::set_error(TV_ERR_INVALID_ARG, "export: grid %d pools blocks of 2^%d voxels (at most 2^24)",
                                 i, lblock);
        tab[(size_t)i] = {r.grid, {ln[0], ln[1], ln[2]}, (r.dims.nz + 31) / 32};
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(ws, tab.data(), sizeof(ExportRef) * tab.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return tv::set_error(TV_ERR_HIP, "export: table upload failed");
    const int64_t total = (int64_t)n << (3 * lres);
    const ExportRef *dtab = static_cast<const ExportRef *>(ws);
    // four cells per thread when they stay within one output row and the
    // output is aligned for a 16-byte (float) or 4-byte (uint8) store
    const bool vec4 = res >= 4 &&
                      (reinterpret_cast<uintptr_t>(out) & (mode == TV_EXPORT_FRACTION ? 15u : 3u)) == 0;
    const int64_t want = (total / (vec4 ? 4 : 1) + kThreads - 1) / kThreads;
    const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
    if (mode == TV_EXPORT_FRACTION) {
        if (vec4) k_export<true, 4><<<blocks, kThreads, 0, s>>>(dtab, total, lres, out);
        else k_export<true, 1><<<blocks, kThreads, 0, s>>>(dtab, total, lres, out);
    } else {
        if (vec4) k_export<false, 4><<<blocks, kThreads, 0, s>>>(dtab, total, lres, out);
        else k_export<false, 1><<<blocks, kThreads, 0, s>>>(dtab, total, lres, out);
    }
    return launched("export launch");
}

}  // extern "C"
