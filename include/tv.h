/*
 * tv.h -- C ABI of the gfx950 tetrahedral-mesh voxelizer.
 *
 * The operation (the paper's voxelization, Section 3 "Voxelization", with the
 * point-in-tet test of Theorem 1, Section 4): for every tetrahedron, every
 * voxel center inside it sets that voxel in a solid binary occupancy grid
 * (the paper voxelizes into a 256^3 binary grid, Table 1).  The library
 * computes this exactly:
 *
 *   - vertices are first placed on a fixed-point lattice of 2^16 units per
 *     bbox extent and per axis (see "Snap" below); all later arithmetic is
 *     exact integer arithmetic on that lattice;
 *   - the sample point of voxel (i,j,k) is its center; with S_a = 2^15 / N_a
 *     the center is ((2i+1)S_x, (2j+1)S_y, (2k+1)S_z) in lattice units;
 *   - a center is inside a tet when all four barycentric coordinates are
 *     positive -- the same decision as Theorem 1's four determinant signs --
 *     and, in TV_TIE_HALF_OPEN mode (the default), a center lying exactly on
 *     a face takes the side it is on after a push by eps*ez + eps^2*ey +
 *     eps^3*ex (eps -> 0+).  In a conforming mesh every center of the union's
 *     interior is then covered exactly once.  TV_TIE_STRICT applies Theorem 1
 *     literally (points on a face are outside), which leaves shared faces
 *     uncovered;
 *   - degenerate (zero-volume) tets add nothing, either vertex orientation is
 *     accepted (Lemma 1.1), overlapping tets give the union.
 *
 * Snap (fp32 input only): per axis a,
 *     q = rint(((double)v - (double)lo[a]) * 65536.0 / ((double)hi[a] - (double)lo[a]))
 * evaluated left to right in IEEE double, round-to-nearest-even, no fused
 * multiply-add.  A NaN or a q outside [TV_Q_MIN, TV_Q_MAX] is a data error.
 *
 * Grid layout: W = ceil(nz/32) uint32 words per (i,j) column; voxel (i,j,k)
 * is bit (k & 31) of word (i*ny + j)*W + (k >> 5).  The whole grid
 * (nx*ny*W words, padding bits included) is overwritten; padding bits are 0.
 *
 * Memory and streams: every data pointer is a DEVICE pointer owned by the
 * caller; the library allocates nothing.  Scratch space is the caller's
 * workspace `ws` of at least the size the matching *_workspace_bytes call
 * returns, aligned to 256 bytes.  Calls are asynchronous on `stream` (a
 * hipStream_t; NULL is the default stream) and return after enqueueing.
 * Calls on different streams with different workspaces may run concurrently;
 * two calls sharing a workspace must be ordered on one stream.  A single-mesh
 * call (tv_voxelize, tv_voxelize_q), tv_batch_run and the grid consumers
 * enqueue kernels only, so they can be captured in a HIP graph and replayed
 * (same pointers and sizes); tv_voxelize_batch and tv_batch_prepare copy the
 * mesh table from host memory and must not be captured.
 *
 * Errors: argument errors that the host can see (null pointers, sizes, dims,
 * bbox, workspace size) return synchronously and enqueue nothing.  Data errors
 * found on the device (a tet index outside [0,nv), a NaN or out-of-range
 * coordinate) are recorded in the workspace; the offending tets are skipped
 * and the grid is still written.  Read them with tv_fetch_status after the
 * work has been enqueued (it synchronizes `stream`).
 */
#ifndef TV_H
#define TV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tv_status;
#define TV_OK 0
#define TV_ERR_INVALID_ARG (-1)      /* null pointer, negative size, bad bbox/flags */
#define TV_ERR_UNSUPPORTED_DIMS (-2) /* a dim that is not a power of two in [1, 32768] */
#define TV_ERR_INDEX (-3)            /* (device) a tet index outside [0, nv) */
#define TV_ERR_RANGE (-4)            /* (device) NaN or coordinate off the lattice range */
#define TV_ERR_WORKSPACE (-5)        /* workspace null, misaligned or too small */
#define TV_ERR_HIP (-7)              /* a HIP runtime call failed */
#define TV_ERR_TOO_LARGE (-8)        /* request larger than the server's memory */
#define TV_ERR_TIMEOUT (-9)          /* wait timed out */
#define TV_ERR_NOT_FOUND (-10)       /* unknown ticket, or result asked before completion */
#define TV_ERR_IO (-11)              /* a mesh file that cannot be read or parsed */

#define TV_Q_MIN (-16384)        /* lattice range: [-2^14, 2^16 + 2^14] per axis */
#define TV_Q_MAX (65536 + 16384)

/* flags */
#define TV_TIE_HALF_OPEN 0u /* default tie rule (see above) */
#define TV_TIE_STRICT 1u    /* Theorem 1 literally: a center on a face is outside */
#define TV_PATH_PER_TET 2u  /* reference path: one lane per tet, word atomics into a
                               cleared grid (same output, slower; for A/B checks) */
#define TV_ACCUMULATE 8u    /* OR the voxels into the grid instead of overwriting it (the
                               grid must hold a previous result or zeros), and keep the
                               data-error status words of earlier calls on this workspace
                               (so a fresh workspace's first call must not accumulate,
                               or come from tv_batch_prepare, which clears them):
                               voxelizing a mesh in several tet subsets gives its grid */

typedef struct {
    int32_t nx, ny, nz; /* each a power of two in [1, 32768] */
} tv_dims;

typedef struct {
    float lo[3], hi[3]; /* world box mapped onto lattice [0, 2^16]; hi > lo per axis */
} tv_bbox;

/* Number of uint32 words of a grid: nx * ny * ceil(nz / 32).  0 for bad dims. */
size_t tv_grid_words(tv_dims dims);

/* Workspace bytes needed by tv_voxelize / tv_voxelize_q for these sizes
 * (about 16 bytes per vertex plus 44 bytes per tet plus a few bytes per
 * grid tile). */
size_t tv_workspace_bytes(int64_t nv, int64_t nt, tv_dims dims, uint32_t flags);

/*
 * Voxelize one mesh given fp32 world coordinates.
 *   verts  [nv][3] float32, device, row-major (x, y, z)
 *   tets   [nt][4] int32, device, vertex indices, 16-byte aligned
 *   dims   grid resolution; bbox: world box covered by the grid
 *   grid   [tv_grid_words(dims)] uint32, device, written entirely
 *   ws     workspace (device, 256-byte aligned, >= tv_workspace_bytes)
 * nt == 0 is valid and yields an all-zero grid.
 */
tv_status tv_voxelize(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                      tv_dims dims, tv_bbox bbox, uint32_t *grid, void *ws, size_t ws_bytes,
                      void *stream, uint32_t flags);

/* As tv_voxelize, with vertices already on the lattice: qverts [nv][3] int32
 * (device), each coordinate in [TV_Q_MIN, TV_Q_MAX]. */
tv_status tv_voxelize_q(const int32_t *qverts, int64_t nv, const int32_t *tets, int64_t nt,
                        tv_dims dims, uint32_t *grid, void *ws, size_t ws_bytes, void *stream,
                        uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tv_voxelize
 * with no workspace argument.  The scratch space is a fixed device array of
 * TV_NOALLOC_MAX_BYTES inside the library, one per GPU, held from the first
 * call on that GPU until the process ends; the call itself allocates nothing.
 *   verts, nv, tets, nt, dims, bbox, grid   as for tv_voxelize
 *   status_out  device int32 (may be NULL): receives the call's data-error
 *               status (TV_OK, TV_ERR_INDEX or TV_ERR_RANGE) on `stream`
 *   flags       0 or TV_TIE_STRICT (nothing else)
 * A mesh whose workspace (tv_workspace_bytes) exceeds TV_NOALLOC_MAX_BYTES
 * (about 1.4 million tets at one vertex per five tets) is refused with TV_ERR_WORKSPACE and nothing is
 * enqueued.  Every call on one GPU shares that GPU's array: calls that
 * overlap on the device (different streams, or different host threads without
 * ordering) race and give undefined results; calls ordered on one stream are
 * safe.  Each call clears the parts of the array it needs zeroed.  The call
 * must be made with the grid's device current.  Like tv_voxelize it enqueues
 * kernels only, so it can be captured in a HIP graph.
 */
#define TV_NOALLOC_MAX_BYTES ((size_t)64 << 20)
tv_status tv_voxelize_noalloc(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                              tv_dims dims, tv_bbox bbox, uint32_t *grid, int32_t *status_out,
                              void *stream, uint32_t flags);

/*
 * Batches: many meshes of uneven size voxelized by one launch sequence
 * (each mesh into its own grid).  `meshes` is a HOST array of n descriptors
 * whose pointers are device pointers; vert_format selects fp32 world
 * coordinates (snapped with the mesh's bbox) or int32 lattice coordinates.
 * Results equal the meshes' single-mesh results bit for bit.  Per-mesh data
 * errors land in status word i (tv_fetch_status(ws, i, stream)) and never
 * affect another mesh.  Host-side argument errors name the offending mesh
 * in tv_last_error() and enqueue nothing.  The descriptor table is copied
 * into the workspace during the call (from pageable host memory; the host
 * array may be reused when the call returns).
 */
#define TV_VERTS_F32 0u
#define TV_VERTS_Q32 1u

typedef struct {
    const void *verts;    /* device [nv][3]: float32 world or int32 lattice */
    uint32_t vert_format; /* TV_VERTS_F32 or TV_VERTS_Q32 */
    int64_t nv;
    const int32_t *tets;  /* device [nt][4] int32, 16-byte aligned */
    int64_t nt;
    tv_dims dims;
    tv_bbox bbox;         /* used with TV_VERTS_F32 */
    uint32_t *grid;       /* device, tv_grid_words(dims) words, written entirely */
} tv_mesh;

size_t tv_batch_workspace_bytes(const tv_mesh *meshes, int32_t n, uint32_t flags);
tv_status tv_voxelize_batch(const tv_mesh *meshes, int32_t n, void *ws, size_t ws_bytes,
                            void *stream, uint32_t flags);

/*
 * The batch call in two steps, for callers that repeat one batch (a HIP
 * graph replay, a loop over fixed device buffers).  The operation is the
 * one above (Section 3: every tet of every mesh, voxel centers tested
 * against it); only the descriptor upload is split off.
 *
 * tv_batch_prepare checks the meshes as tv_voxelize_batch does, copies their
 * descriptor table into `ws` and clears the meshes' status words
 * (asynchronously on `stream`: a copy from pageable host memory, so `meshes`
 * may be reused when it returns, and a memset; no kernel), and fills *plan,
 * a small host struct owned by the caller.  Runs of a plan prepared with
 * TV_ACCUMULATE therefore report the data errors of every run since the
 * prepare.
 * TV_PATH_PER_TET is rejected (TV_ERR_INVALID_ARG).
 *
 * tv_batch_run enqueues the batch's kernels on `stream` and nothing else: no
 * host copies, memsets or allocations, so a run can be captured in a HIP
 * graph and replayed (with stage profiling off while capturing).  Each run
 * voxelizes the current contents of the meshes' vertex and tet buffers into
 * their grids, bit for bit as tv_voxelize_batch, with the flags given to
 * tv_batch_prepare; status words as for tv_voxelize_batch.  `ws` must be
 * the workspace the plan was prepared in (else TV_ERR_INVALID_ARG), still
 * holding the table: any other call that uses `ws` in between overwrites
 * it, and the batch must then be prepared again.  A plan not filled by
 * tv_batch_prepare, or edited, is rejected with TV_ERR_INVALID_ARG.  Runs
 * sharing one workspace must be ordered on one stream.
 */
typedef struct {
    int64_t meshes, nv, nt, ntiles; /* totals of the prepared batch */
    uint64_t ws;                    /* address of the workspace holding the table */
    uint32_t flags;                 /* flags given to tv_batch_prepare */
    int32_t launch[5];              /* launch parameters in force at prepare time */
    uint32_t check;                 /* consistency tag */
} tv_batch_plan;

tv_status tv_batch_prepare(const tv_mesh *meshes, int32_t n, void *ws, size_t ws_bytes,
                           void *stream, uint32_t flags, tv_batch_plan *plan);
tv_status tv_batch_run(const tv_batch_plan *plan, void *ws, size_t ws_bytes, void *stream);

/*
 * Launch parameters of the tile pipeline, one set for single-mesh calls
 * (tv_voxelize, tv_voxelize_q, tv_voxelize_pipelined) and one for batch
 * calls.  They change speed only: every valid setting gives the same grids
 * bit for bit.  (They are this library's work decomposition, not the
 * paper's: Section 3 tests each tet's bounding-box candidates, and every
 * setting still does exactly that.)
 *   tile_cols_log2  largest tile edge in columns, log2, in [3, 5]
 *   min_tiles       tiles are halved (down to 8 x 8 columns) while a grid
 *                   has fewer than this, in [1, 2^20]
 *   chunk_pieces    (tet, tile) pieces per work-queue task, in [64, 65536];
 *                   0 picks, for one mesh, about nt / 2048 (a power of two
 *                   in [256, 16384]; at least 4096 when the call has 4096
 *                   tiles or more), for a batch about nt / 1024 (a power of
 *                   two in [256, 65536])
 *   strip_columns   kept columns per lane task, in [1, 64]
 *   piece_cap       tets meeting more tiles take the per-tet large path, [1, 8]
 *   wgs_per_cu      persistent tile workgroups per compute unit, in [1, 8]
 *   cull_columns    a piece whose clipped box has at most this many columns
 *                   skips the per-row culling by its xy hull, in [0, 1024]
 * Defaults (tv_default_params): single {5, 512, 0, 6, 8, 2, 3}, batch
 * {5, 1, 0, 6, 8, 2, 6}.  tv_set_params validates all fields
 * (TV_ERR_INVALID_ARG, nothing changed) and with p == NULL restores the
 * defaults.  The settings are process-wide; each call copies them when it
 * starts, so set them before enqueueing work.  Workspace sizes depend on
 * the tile fields: query tv_*_workspace_bytes after a change.  A prepared
 * batch keeps the parameters of its tv_batch_prepare call.  The server
 * always uses the batch defaults.  The autotuner that picks them lives in
 * the Python package (timings on the device, a JSON cache).
 */
typedef struct {
    int32_t tile_cols_log2, min_tiles, chunk_pieces, strip_columns, piece_cap, wgs_per_cu,
        cull_columns;
} tv_params;
#define TV_PARAMS_SINGLE 0
#define TV_PARAMS_BATCH 1
tv_status tv_default_params(int32_t which, tv_params *out);
tv_status tv_get_params(int32_t which, tv_params *out);
tv_status tv_set_params(int32_t which, const tv_params *p);

/*
 * Snap only: fp32 world coordinates verts [nv][3] -> lattice coordinates
 * q_out [nv][3] int32 (both device), per the snap rule above.  A vertex that
 * is NaN or off the lattice range is written as three TV_Q_INVALID values.
 * Asynchronous on `stream`; argument errors as for tv_voxelize.
 */
#define TV_Q_INVALID INT32_MIN
tv_status tv_snap(const float *verts, int64_t nv, tv_bbox bbox, int32_t *q_out, void *stream);

/*
 * Data-error status of mesh `mesh_index` recorded in workspace `ws` by the
 * last call that used it (index 0 for the single-mesh calls, the mesh's
 * position for a batch).  Synchronizes `stream`, then returns TV_OK,
 * TV_ERR_INDEX or TV_ERR_RANGE (TV_ERR_INDEX wins when both occurred), or
 * TV_ERR_INVALID_ARG (index outside the last call's meshes) / TV_ERR_HIP.
 * After tv_voxelize_bricks it also reports TV_ERR_TOO_LARGE (brick pool
 * too small), after the other two.
 */
tv_status tv_fetch_status(const void *ws, int32_t mesh_index, void *stream);

/*
 * Diagnostics: per-stage timing with HIP events.  While enabled, every call
 * records a start and an end event around each of its stages on its own
 * stream.  tv_profile_read waits for those events, returns the summed
 * milliseconds per stage (ms_out[stage], up to max_stages entries) and the
 * number of calls recorded, then clears the record.  Process-wide state; not
 * meant for concurrent callers.  Stage names: tv_profile_stage_name.
 */
tv_status tv_profile_enable(int32_t on);
tv_status tv_profile_read(double *ms_out, int32_t max_stages, int32_t *n_stages, int64_t *n_calls);
const char *tv_profile_stage_name(int32_t stage);

/*
 * Serving: a continuous-batching server for voxelization requests (the
 * paper's observation that for small models transfer and allocation cost
 * more than the voxelization itself, Section 3 "Parallelization" and
 * Table 1, is why requests are batched and memory is kept allocated).
 *
 *   - tv_server_create allocates, once, a device arena (inputs, grids and
 *     wave workspaces live in it) and a pinned host staging area, creates
 *     `streams` compute streams and starts, on the current device, a
 *     scheduler thread, one launcher thread per stream (it stages host
 *     inputs and enqueues the wave's copies and kernels, so admission never
 *     waits for a copy) and a completion thread.
 *   - tv_server_submit queues a request (host or device inputs, see flags);
 *     the scheduler admits queued requests in FIFO order while their memory
 *     footprint (inputs + grid + workspace share) fits in the arena and a
 *     stream is free, groups them into a wave (one batched launch sequence,
 *     tv_voxelize_batch semantics) and launches it; requests that arrive
 *     while other waves run are admitted into the next wave as soon as a
 *     stream and memory free up, so waves overlap on the device.
 *   - A request's grid stays in device memory after completion until
 *     tv_server_release; tv_server_result gives its device address, and its
 *     latency (completion - submission, host steady clock).
 *   - All calls are thread-safe; results equal tv_voxelize's bit for bit.
 */
typedef struct tv_server tv_server;

#define TV_REQ_HOST_INPUTS 0u   /* verts/tets in pageable host memory: staged through pinned memory */
#define TV_REQ_PINNED_INPUTS 4u /* verts/tets in pinned host memory: copied directly */
#define TV_REQ_DEVICE_INPUTS 8u /* verts/tets already in device memory: not copied */

typedef struct {
    const void *verts;     /* [nv][3] float32 world or int32 lattice (vert_format) */
    uint32_t vert_format;  /* TV_VERTS_F32 or TV_VERTS_Q32 */
    int64_t nv;
    const int32_t *tets;   /* [nt][4] int32 */
    int64_t nt;
    tv_dims dims;
    tv_bbox bbox;
    uint32_t flags;        /* TV_TIE_STRICT | one TV_REQ_*_INPUTS; inputs must stay valid
                              until the request is done */
} tv_request;

typedef struct {
    size_t device_bytes;      /* device arena */
    size_t pinned_bytes;      /* pinned host staging (0: pageable inputs are refused) */
    int32_t streams;          /* waves in flight at once (>= 1) */
    int32_t max_wave_meshes;  /* meshes per wave (>= 1) */
} tv_server_config;

typedef struct {
    int64_t submitted, completed, released, rejected;
    int64_t waves;            /* waves launched */
    int64_t queued;           /* requests waiting for admission */
    int64_t running;          /* requests in waves on the device */
    int64_t inflight_waves;
    size_t device_in_use, device_peak, pinned_in_use;
    int64_t inflight_peak;    /* most waves in flight at once so far */
} tv_server_stats;

#define TV_REQ_QUEUED 0
#define TV_REQ_RUNNING 1
#define TV_REQ_DONE 2

tv_status tv_server_create(const tv_server_config *cfg, tv_server **out);
/* Queues a request; TV_ERR_TOO_LARGE when it could never fit. */
tv_status tv_server_submit(tv_server *s, const tv_request *req, int64_t *ticket);
tv_status tv_server_poll(tv_server *s, int64_t ticket, int32_t *state);
/* Blocks until the request is done (TV_ERR_TIMEOUT after timeout_s > 0). */
tv_status tv_server_wait(tv_server *s, int64_t ticket, double timeout_s);
/* Done request: device grid address and word count, the request's data
 * status (TV_OK / TV_ERR_INDEX / TV_ERR_RANGE) and latency in seconds. */
tv_status tv_server_result(tv_server *s, int64_t ticket, const uint32_t **grid, size_t *words,
                           tv_status *data_status, double *latency_s);
/* Copies a done request's grid to `dst` (host or device memory; blocking). */
tv_status tv_server_copy_grid(tv_server *s, int64_t ticket, void *dst, size_t words);
/* Frees a done request's grid. */
tv_status tv_server_release(tv_server *s, int64_t ticket);
tv_status tv_server_get_stats(tv_server *s, tv_server_stats *out);
/* Waits for in-flight waves, stops the threads and frees everything. */
tv_status tv_server_destroy(tv_server *s);

/*
 * Voxelization from host inputs with the copies overlapped (the transfer
 * cost of Table 1's CPU+GPU column): the vertices, then the tets in `chunks`
 * consecutive slices, are copied on `copy_stream` into the caller's device
 * buffers verts_dev [nv][3] and tets_dev [nt][4]; on `stream`, slice k is
 * voxelized as soon as it has arrived (slice 0 overwrites the grid, later
 * slices use TV_ACCUMULATE), so copying slice k+1 overlaps voxelizing slice
 * k.  The grid equals tv_voxelize's on the whole mesh.  Host inputs should
 * be pinned for the copies to run asynchronously.  `ws` needs
 * tv_workspace_bytes(nv, ceil(nt / chunks), dims, flags) bytes.  chunks is
 * clamped to [1, 64]; every slice repeats the launch sequence (and the snap
 * of all vertices), so slices of about a million tets or more pay off.  With
 * one slice the copies simply run on `stream`.  The library keeps a small pool
 * of HIP events per calling thread and device for the slices.  Returns after
 * enqueueing; `stream` orders after all the copies.  flags: TV_TIE_STRICT,
 * TV_PATH_PER_TET.
 */
tv_status tv_voxelize_pipelined(const float *verts_host, int64_t nv, const int32_t *tets_host,
                                int64_t nt, tv_dims dims, tv_bbox bbox, float *verts_dev,
                                int32_t *tets_dev, uint32_t *grid, void *ws, size_t ws_bytes,
                                void *stream, void *copy_stream, int32_t chunks, uint32_t flags);

/*
 * Grid consumers (device-side, asynchronous on `stream`, allocate nothing).
 * The paper motivates solid grids by 3D CNN training data (Section 1; the
 * 3D CNN connection itself is left to future work in Section 6) and notes
 * that the sparse nature of voxel data favours sparse storage (Octrees
 * paragraph, Section 5).  These calls turn a packed grid (layout above)
 * into what such consumers read.
 *
 * tv_unpack: dense tensor out[nx][ny][nz] (z fastest, C order) with 1 for a
 *   set voxel and 0 otherwise; TV_UNPACK_U8 writes uint8, TV_UNPACK_F32
 *   float32.  `out` holds nx*ny*nz elements (16-byte alignment selects the
 *   vectorized path; any alignment of the element type is accepted).
 *   Errors: TV_ERR_UNSUPPORTED_DIMS, TV_ERR_INVALID_ARG (null, format).
 */
#define TV_UNPACK_U8 0u
#define TV_UNPACK_F32 1u
tv_status tv_unpack(const uint32_t *grid, tv_dims dims, void *out, uint32_t format, void *stream);

/*
 * tv_pool: a coarser level by `factor` f (a power of two in [2, 32] that
 * divides nx, ny and nz); output dims (nx/f, ny/f, nz/f).
 *   TV_POOL_FRACTION: float32 out[nx/f][ny/f][nz/f] = (set voxels of the
 *     f^3 block) / f^3, a multiple of 2^-15 computed exactly;
 *   TV_POOL_ANY: a packed grid of dims / f (same layout, padding bits 0)
 *     whose voxel is set iff any voxel of its block is.
 *   Errors: TV_ERR_UNSUPPORTED_DIMS, TV_ERR_INVALID_ARG (factor, mode, null).
 */
#define TV_POOL_FRACTION 0u
#define TV_POOL_ANY 1u
tv_status tv_pool(const uint32_t *grid, tv_dims dims, int32_t factor, uint32_t mode, void *out,
                  void *stream);

/*
 * tv_export_batch: many grids of any dims (for instance the grids of one
 * tv_voxelize_batch call) into ONE dense tensor out[n][res][res][res] (C
 * order, z fastest) for a 3D CNN, in one kernel launch.  Per axis, a grid
 * finer than res is pooled by n_a / res and a coarser one repeats each voxel
 * res / n_a times, so every grid lands at the common resolution res.  The
 * value of a cell, from its source block (the voxels it pools, or the one
 * voxel it repeats):
 *   TV_EXPORT_FRACTION: float32, set voxels of the block / voxels of the
 *     block (exact: a multiple of a power of two);
 *   TV_EXPORT_ANY: uint8, 1 when any voxel of the block is set.
 * `grids` is a HOST array of n (device grid pointer, dims) pairs; it is
 * copied into `ws` (device, 256-byte aligned, tv_export_workspace_bytes(n)
 * bytes) during the call, so the call must not be captured in a graph.
 * res: a power of two in [1, 1024]; a pooled block may hold at most 2^24
 * voxels.  Errors: TV_ERR_INVALID_ARG (null, n, res, mode, block size),
 * TV_ERR_UNSUPPORTED_DIMS (a grid's dims), TV_ERR_WORKSPACE.
 */
typedef struct {
    const uint32_t *grid; /* device, packed layout above */
    tv_dims dims;
} tv_grid_ref;
#define TV_EXPORT_FRACTION 0u
#define TV_EXPORT_ANY 1u
size_t tv_export_workspace_bytes(int32_t n);
tv_status tv_export_batch(const tv_grid_ref *grids, int32_t n, int32_t res, uint32_t mode, void *out,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * tv_voxelize_bricks: voxelize one mesh (fp32 world coordinates, as
 * tv_voxelize) straight into sparse bricks, with no dense grid -- for grids
 * whose dense form is not worth keeping (a 4096^3 grid is 8 GiB; the paper's
 * Octrees paragraph, Section 5, discusses sparse storage of such data).  A
 * brick is 8 x 8 columns by 32 z voxels, laid out as in tv_bricks below:
 * brick (bx, by, bz) has id (bx*(ny/8) + by)*(nz/32) + bz and word u*8 + v
 * of a brick is word bz of column (8bx+u, 8by+v).  Outputs (device, owned by
 * the caller):
 *   index     [tv_brick_count_max(dims)] uint32, written entirely: 0 for an
 *             empty brick, TV_BRICK_FULL when every voxel of the brick is
 *             set, otherwise 1 + the brick's slot in pool;
 *   pool      [capacity][64] uint32: the words of the slotted bricks;
 *   pool_ids  [capacity] uint32: the brick id of each slot, or
 *             TV_BRICK_UNUSED for a slot given up (several writers can race
 *             for a brick; the losers merge into the winner's slot);
 *   pool_count one uint32: the slots taken, including given-up ones.
 * A brick is in the pool iff it is neither empty nor full, so the bricks are
 * unique; their slot order is not.  Each tile of the grid is voxelized by
 * one workgroup, so the slots taken are the pooled bricks plus the few given
 * up where two tets too large for the tile pipeline race for a new brick.
 * If pool_count exceeds capacity the output is incomplete and the data-error
 * status (tv_fetch_status(ws, 0, stream)) reads TV_ERR_TOO_LARGE: call again
 * with capacity >= pool_count.
 * dims: powers of two with nx, ny >= 8 and nz >= 32, at most 2^32 - 2
 * bricks.  ws: tv_voxelize_bricks_workspace_bytes(nv, nt, dims) bytes (the
 * dense call's workspace with room for up to 27 tiles per tet, about 16
 * bytes per vertex plus 120 per tet).  flags: 0 or TV_TIE_STRICT.  Enqueues
 * kernels only (graph-capturable).
 */
#define TV_BRICK_FULL 0xffffffffu
#define TV_BRICK_UNUSED 0xffffffffu
size_t tv_voxelize_bricks_workspace_bytes(int64_t nv, int64_t nt, tv_dims dims);
tv_status tv_voxelize_bricks(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                             tv_dims dims, tv_bbox bbox, uint32_t *index, uint32_t *pool,
                             uint32_t *pool_ids, int64_t capacity, uint32_t *pool_count, void *ws,
                             size_t ws_bytes, void *stream, uint32_t flags);

/*
 * tv_bricks: the non-empty bricks of a grid, in increasing brick id.  A
 * brick is 8 x 8 columns by 32 z voxels -- one grid word per column, 256
 * bytes; brick (bx, by, bz) has id (bx*(ny/8) + by)*(nz/32) + bz and its
 * 64 words are those of columns (8bx+u, 8by+v), u, v in [0, 8), word bz,
 * u-major.  Needs nx, ny multiples of 8 and nz of 32 (else
 * TV_ERR_UNSUPPORTED_DIMS); tv_brick_count_max gives the number of bricks
 * (0 for such dims).  Writes the number of non-empty bricks to the device
 * word `count`, and the first min(count, capacity) of them to ids[] and
 * brick_words[] (64 words each, 16-byte aligned); capacity 0 only counts.
 * `ws` (device) holds tv_bricks_workspace_bytes(dims) bytes of scratch.
 */
int64_t tv_brick_count_max(tv_dims dims);
size_t tv_bricks_workspace_bytes(tv_dims dims);
tv_status tv_bricks(const uint32_t *grid, tv_dims dims, uint32_t *ids, uint32_t *brick_words,
                    int64_t capacity, uint32_t *count, void *ws, size_t ws_bytes, void *stream);

/*
 * Tet-mesh files (host side; the step before voxelization: the paper's
 * pipeline voxelizes the tetrahedral meshes its mesher writes, Section 3).
 * tv_read_mesh parses a MEDIT ".mesh" (ASCII; Dimension 3, sections
 * Vertices and Tetrahedra, other known sections skipped) or a Gmsh ".msh"
 * file (ASCII, format 2.2 or 4.1; 4-node tetrahedra, other element types
 * skipped), detected from the file's first token.  Coordinates are parsed as
 * double and rounded to float; tet indices become 0-based.  On success the
 * library allocates `verts` [nv][3] and `tets` [nt][4] in host memory (free
 * them with tv_free_host_mesh) and sets bbox to the vertices' min/max.
 * Errors: TV_ERR_INVALID_ARG, TV_ERR_IO (unreadable, malformed, binary or
 * unsupported content, an index to an unknown vertex); nothing is allocated
 * then.
 */
typedef struct {
    float *verts;               /* [nv][3] */
    int64_t nv;
    int32_t *tets;              /* [nt][4], 0-based */
    int64_t nt;
    tv_bbox bbox;               /* min / max of the vertices */
    int64_t skipped_elements;   /* elements that are not 4-node tetrahedra */
} tv_host_mesh;
tv_status tv_read_mesh(const char *path, tv_host_mesh *out);
void tv_free_host_mesh(tv_host_mesh *m);

/*
 * Mesh quality report: the assumptions the paper's voxelizer makes about its
 * input (Section 3, "Voxelization": a large minimum angle, no overlapping
 * tets, small variance), measured on the voxelizer's own lattice.  Inputs
 * as for tv_voxelize (vert_format TV_VERTS_F32 with bbox, or TV_VERTS_Q32
 * lattice coordinates, in which case bbox only scales lattice units to
 * world units), plus `grid`: the grid of these tets at `dims` (device; e.g.
 * what tv_voxelize wrote).  `flags` may hold TV_TIE_STRICT.  Blocking: it
 * synchronizes `stream` and fills the host struct `out`.
 *   tets / invalid: tets examined / skipped for an index outside [0, nv) or
 *     a vertex that fails to snap (or lies off the lattice range);
 *   degenerate / inverted: 6V == 0 / 6V < 0 on the lattice (exact);
 *   min_dihedral_deg, mean_min_dihedral_deg, min_dihedral_below[k]: over
 *     non-degenerate tets, the smallest of a tet's six dihedral angles in
 *     world coordinates (degrees): its minimum, its mean, and how many tets
 *     have it below 1, 5, 10 and 20 degrees;
 *   volume_mean, volume_cv: mean and coefficient of variation (std / mean)
 *     of the non-degenerate tets' volumes (world units);
 *   covered_voxels: the sum over tets of the voxel centers each contains
 *     under the voxelizer's rule; occupied_voxels: set voxels of `grid`.
 *     Without overlapping tets the two are equal (exactly, under the
 *     half-open rule); covered - occupied counts the extra coverage.
 * `ws` (device, 256-byte aligned) holds tv_quality_workspace_bytes(nv).
 */
typedef struct {
    int64_t tets, invalid, degenerate, inverted;
    int64_t min_dihedral_below[4]; /* below 1, 5, 10, 20 degrees */
    double min_dihedral_deg, mean_min_dihedral_deg;
    double volume_mean, volume_cv;
    int64_t covered_voxels, occupied_voxels;
} tv_quality;
size_t tv_quality_workspace_bytes(int64_t nv);
tv_status tv_mesh_quality(const void *verts, uint32_t vert_format, int64_t nv, const int32_t *tets,
                          int64_t nt, tv_dims dims, tv_bbox bbox, const uint32_t *grid, uint32_t flags,
                          void *ws, size_t ws_bytes, void *stream, tv_quality *out);

/* Human-readable name of a status code (static storage). */
const char *tv_status_string(tv_status s);

/* Message of the last error returned on the calling thread (thread-local). */
const char *tv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TV_H */
