/*
 * cga.h -- C ABI of the MI355X (gfx950) compressed-geometric-array library.
 *
 * A compressed geometric array (CGA, Section V of "Compressed Geometric
 * Arrays for Point Cloud Processing") stores the occupied voxels of a point
 * cloud in ascending (x, y, z) order with the x and (x, y) prefixes run-length
 * encoded.  This library keeps the same set as one sorted array of unique
 * voxel keys -- LINEAR keys x<<2d | y<<d | z give exactly the paper's order,
 * MORTON keys interleave the bits (x most significant within each bit
 * triple) for octree locality -- and derives the paper's five coordinate
 * arrays from it on demand (cga_to_arrays).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are device pointers owned by the caller; h_* and
 *    *_host pointers are host pointers.  The library never allocates or frees
 *    device memory; calls that need scratch space take a caller-owned
 *    workspace (d_ws, ws_bytes) whose minimum size the matching
 *    *_workspace_bytes function returns (one call, cga_merge_noalloc, uses
 *    a static device array of the library instead).  A workspace may be
 *    reused by later calls on the same stream, never by two calls in flight
 *    at once.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and the call returns without waiting, unless a *_host output pointer is
 *    non-NULL: then the call synchronises the stream, fills it, and also
 *    returns any error the device detected.
 *  - Key arrays are uint32 when 3*depth <= 32 and uint64 otherwise
 *    (cga_key_bytes); 2-D pixel keys are uint32 when 2*depth <= 32.
 *  - Counts may live on the device: every array input has a host size n (an
 *    upper bound, used to size launches) and an optional d_n (device int64
 *    holding the actual size <= n).  Outputs report their size through an
 *    optional d_n_out (device int64) and n_out_host.  This lets a whole
 *    pipeline run, or be captured in a hipGraph, without host round trips.
 *  - Device-detected errors (non-finite coordinates, an output larger than its
 *    capacity) are recorded in the first word of the workspace; n_out_host
 *    callers get them as the return value, others call cga_ws_status.
 *    After CGA_ECAPACITY the output contents are unspecified.
 *  - Return value: CGA_OK or a negative cga_status.  Arguments are validated
 *    on the host before anything is enqueued.
 *  - Sizes: n < 2^31 per array.
 */
#ifndef CGA_H
#define CGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *cga_stream; /* hipStream_t */

enum cga_status {
    CGA_OK = 0,
    CGA_EINVAL = -1,       /* bad argument (depth, k, axis, null pointer, n < 0 ...) */
    CGA_ECAPACITY = -2,    /* an output exceeded the capacity the caller gave */
    CGA_EMISMATCH = -3,    /* operands disagree (grid / key width / index header) */
    CGA_ENONFINITE = -4,   /* a NaN or Inf coordinate */
    CGA_EHIP = -5,         /* a HIP runtime error; see cga_last_hip_error */
    CGA_EWORKSPACE = -6,   /* workspace smaller than required */
    CGA_EUNSUPPORTED = -7  /* valid request this build does not implement */
};

enum cga_key_mode { CGA_KEY_MORTON = 0, CGA_KEY_LINEAR = 1 };

/* Quantization frame.  Per axis a: voxel_a = clamp(floor(fl32(fl32(p_a -
 * origin_a) * scale)), 0, 2^depth - 1), subtract and multiply each rounded
 * to nearest float32 (never fused).  The cubic bounding box of all clouds
 * that will be combined is the usual frame (Section II-E, bounding-box
 * alignment); the paper's own data is already integer voxels (Table II).
 * depth in [1, 21]; scale finite and > 0; origin finite. */
typedef struct {
    float origin[3];
    float scale;
    uint32_t depth;
    uint32_t key_mode; /* cga_key_mode */
} cga_grid;

/* Optional launch tuning (NULL = built-in or autotuned defaults).  Never
 * changes results.  radix_bits in [4, 11]; tile_items in {8, 12, 16, 24, 32}. */
typedef struct {
    uint32_t radix_bits;
    uint32_t tile_items;
} cga_tune;

/* ---------------------------------------------------------------- helpers */
const char *cga_strerror(int status);
int cga_last_hip_error(void);
size_t cga_key_bytes(const cga_grid *grid);  /* 4 or 8; 0 for an invalid grid */
size_t cga_key2_bytes(const cga_grid *grid); /* 2-D pixel key width */
/* Synchronise `stream` and return the error recorded in d_ws by the last
 * call that used it (CGA_OK if none). */
int cga_ws_status(const void *d_ws, cga_stream stream);

/* ------------------------------------------------------------------ build
 * CGA construction (Section V): quantize n float32 points (AoS x,y,z) by
 * the grid rule, encode each voxel as a key, radix-sort the keys and collapse
 * equal keys.  Output: the U unique keys ascending in d_keys (capacity cap)
 * and, if d_counts is non-NULL, the number of input points in each voxel
 * (uint32).  U goes to d_n_out / n_out_host.  n may be 0.
 * Errors: CGA_ENONFINITE (device), CGA_ECAPACITY if U > cap (device). */
size_t cga_build_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_build(const cga_grid *grid, const float *d_xyz, int64_t n, void *d_keys,
              uint32_t *d_counts, int64_t cap, int64_t *d_n_out, int64_t *n_out_host,
              void *d_ws, size_t ws_bytes, const cga_tune *tune, cga_stream stream);

/* Quantize + encode only: the per-point key of each input point, in input
 * order (no sort, no dedupe).  Exposed for parity tests of the encoder. */
int cga_encode_keys(const cga_grid *grid, const float *d_xyz, int64_t n, void *d_keys,
                    void *d_ws, size_t ws_bytes, cga_stream stream);

/* Stable LSD radix sort of n keys of the grid's key width on their low
 * `key_bits` bits (the significant bits of the grid's keys if 0).  Sorted
 * keys go to d_out (may equal d_keys).  Exposed for parity tests. */
size_t cga_sort_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_sort_keys(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint32_t key_bits, void *d_out, void *d_ws, size_t ws_bytes,
                  const cga_tune *tune, cga_stream stream);

/* The paper's five CGA arrays (Section V) from a LINEAR-mode key array of n
 * unique ascending keys.  Readings of the definitions: all levels ascending;
 * X_pointer is indexed by position in X_index (length n_x + 1) and counts the
 * distinct y of each x; Y_pointer counts the z of each (x, y) pair (length
 * n_xy + 1).  Outputs (capacity n each, pointers n + 1): d_x_index (uint32),
 * d_x_ptr (int64), d_y_index (uint32), d_y_ptr (int64), d_z_index (uint32);
 * n_x and n_xy go to the optional device/host outputs.
 * CGA_EMISMATCH for a MORTON grid. */
size_t cga_to_arrays_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_to_arrays(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint32_t *d_x_index, int64_t *d_x_ptr, uint32_t *d_y_index, int64_t *d_y_ptr,
                  uint32_t *d_z_index, int64_t *d_n_x, int64_t *d_n_xy, int64_t *n_x_host,
                  int64_t *n_xy_host, void *d_ws, size_t ws_bytes, cga_stream stream);

/* ------------------------------------------------- paper's array operations
 * The paper's own algorithms on the five arrays of a LINEAR grid, as
 * cga_to_arrays writes them: n_x entries of X_index (X_pointer has n_x + 1),
 * n_xy of Y_index (Y_pointer n_xy + 1), n of Z_index.  d_n_x / d_n_xy are
 * optional device counts (at most the host bounds), so that the arrays can
 * stay on the device.  Pointer entries outside those lengths raise
 * CGA_EMISMATCH (device) and are clamped, so every access stays in bounds.
 * CGA_EMISMATCH (host) for a MORTON grid.  Workspace:
 * cga_arrays_ops_workspace_bytes() bytes (the call's error block). */
size_t cga_arrays_ops_workspace_bytes(void);

/* Point lookup, Section V-A: for each of nq query voxels (uint32 x, y, z,
 * AoS) the three-level search -- x in X_index, y in that x's run of
 * Y_index (bounded by X_pointer, indexed by the x's position), z in that
 * (x, y)'s run of Z_index (bounded by Y_pointer).  d_pos[j] = the voxel's
 * position in Z_index, which is the index of its LINEAR key, or -1 when it
 * is absent (also for coordinates outside the grid). */
int cga_arrays_lookup(const cga_grid *grid, const uint32_t *d_x_index, int64_t n_x,
                      const int64_t *d_n_x, const int64_t *d_x_ptr, const uint32_t *d_y_index,
                      int64_t n_xy, const int64_t *d_n_xy, const int64_t *d_y_ptr,
                      const uint32_t *d_z_index, int64_t n, const uint32_t *d_qvox, int64_t nq,
                      int64_t *d_pos, void *d_ws, size_t ws_bytes, cga_stream stream);

/* Nearest neighbour, Section V-C: each of nq float32 query points (AoS) is
 * quantized by the grid rule; the nearest x, then y, then z give a first
 * point at distance epsilon, and the closest point within epsilon of the
 * query on every axis is the answer: the same voxel as cga_knn with k = 1
 * (ties to the smaller key).  d_idx = its position in Z_index (-1 for an
 * empty CGA), d_d2 = its squared voxel distance (UINT64_MAX when none).
 * Errors: CGA_ENONFINITE for a non-finite query (device). */
int cga_arrays_nn(const cga_grid *grid, const uint32_t *d_x_index, int64_t n_x,
                  const int64_t *d_n_x, const int64_t *d_x_ptr, const uint32_t *d_y_index,
                  int64_t n_xy, const int64_t *d_n_xy, const int64_t *d_y_ptr,
                  const uint32_t *d_z_index, int64_t n, const float *d_q, int64_t nq,
                  int64_t *d_idx, uint64_t *d_d2, void *d_ws, size_t ws_bytes, cga_stream stream);

/* ---------------------------------------------------- temporal prediction
 * One inter-frame step of the CGA point cloud compression scheme (Section
 * V-D): a predicted frame against a reference frame, both CGAs of the same
 * grid (ascending unique keys of the grid's width and mode, one packed
 * 4 x 8-bit value per voxel, as cga_voxel_values writes them).
 *   1. k-means over each frame's voxels with eight centres started at the
 *      corners of its bounding box (centre i: maximum x if bit 2 of i is
 *      set, else minimum; y by bit 1; z by bit 0).  A pass assigns every
 *      voxel to its nearest centre (squared distance in double precision,
 *      (dx^2 + dy^2) + dz^2 with every operation rounded, ties to the lower
 *      centre); the run ends at the first pass that changes no assignment,
 *      or after max_iter passes, else each non-empty cluster moves to its
 *      mean (exact integer sums, one rounded division).
 *   2. motion vector of cluster i: predicted minus reference centroid i,
 *      rounded half away from zero to whole voxels.
 *   3. each predicted voxel moved back by its cluster's vector is matched to
 *      the reference voxel of least SAD over the four channels among those
 *      within `window` voxels on every axis (ties: smaller L1 offset, then
 *      smaller key).
 *   4. residual = predicted minus matched channels, as int16.
 * Outputs: d_ref_assign / d_pred_assign (uint8 cluster per voxel), optional
 * d_centroids (double [2][8][3]: reference, predicted), d_mv (int32 [8][3]),
 * d_iters (int32 [2]: passes run), d_match (int64 index into the reference
 * keys, -1 when the moved voxel left the grid or its window holds no
 * reference voxel), d_sad (uint32, UINT32_MAX without a match), d_residual
 * (int16 [n_pred][4]; the voxel's own channels without a match).
 * window in [0, 15], max_iter in [1, 1000] (else CGA_EINVAL).  The keys
 * are trusted to be sorted and unique.  Workspace:
 * cga_temporal_workspace_bytes() bytes. */
size_t cga_temporal_workspace_bytes(void);
int cga_temporal_predict(const cga_grid *grid, const void *d_ref_keys, const uint32_t *d_ref_values,
                         int64_t n_ref, const void *d_pred_keys, const uint32_t *d_pred_values,
                         int64_t n_pred, int window, int max_iter, uint8_t *d_ref_assign,
                         uint8_t *d_pred_assign, double *d_centroids, int32_t *d_mv,
                         int32_t *d_iters, int64_t *d_match, uint32_t *d_sad, int16_t *d_residual,
                         void *d_ws, size_t ws_bytes, cga_stream stream);

/* ------------------------------------------------------------------ merge
 * Merge, Eq. (1): the union of two CGAs of the same grid (sorted unique key
 * arrays a, b) as one sorted unique key array.  d_src (nullable) receives a
 * provenance byte per output key: 1 = only in a, 2 = only in b, 3 = both.
 * Errors: CGA_ECAPACITY if the union exceeds cap (device). */
size_t cga_merge_workspace_bytes(const cga_grid *grid, int64_t na, int64_t nb);
int cga_merge(const cga_grid *grid, const void *d_a, int64_t na, const int64_t *d_na,
              const void *d_b, int64_t nb, const int64_t *d_nb, void *d_out, uint8_t *d_src,
              int64_t cap, int64_t *d_n_out, int64_t *n_out_host, void *d_ws, size_t ws_bytes,
              cga_stream stream);

/* The same merge with no workspace argument and no allocation, for callers
 * that cannot allocate device memory (code under hipGraph capture, serving
 * loops, harnesses that forbid hipMalloc).  Its scratch space is a static
 * device array of the library (about 2 MiB, one copy per GPU, held until the
 * process ends), found for the current device on its first call there; the
 * current device must be the stream's.  Inputs, outputs and results are as
 * for cga_merge.  na + nb above CGA_MERGE_NOALLOC_MAX_KEYS: CGA_EWORKSPACE,
 * before anything is enqueued.  Every call on one GPU shares that array:
 * calls that overlap in time on one GPU (two streams, two host threads) race
 * and give undefined results; calls in stream order are safe.  Device errors
 * (CGA_ECAPACITY) come back only through n_out_host (and a device count above
 * cap in d_n_out). */
#define CGA_MERGE_NOALLOC_MAX_KEYS ((int64_t)1 << 28)
int cga_merge_noalloc(const cga_grid *grid, const void *d_a, int64_t na, const int64_t *d_na,
                      const void *d_b, int64_t nb, const int64_t *d_nb, void *d_out,
                      uint8_t *d_src, int64_t cap, int64_t *d_n_out, int64_t *n_out_host,
                      cga_stream stream);

/* ------------------------------------------------------------- projection
 * Orthogonal projection, Eq. (3) with m_x = m_y = 1 (Section V-B), along
 * axis drop_axis (0 = x, 1 = y, 2 = z): the set of 2-D pixels (u, v) -- the
 * two remaining coordinates in x, y, z order -- hit by at least one voxel, as
 * sorted unique 2-D keys (MORTON: u bit b -> 2b+1, v bit b -> 2b; LINEAR:
 * u<<d | v), with the number of voxels on each pixel in d_counts (nullable).
 * Errors: CGA_ECAPACITY (device). */
size_t cga_project_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_project(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
                int drop_axis, void *d_out2d, uint32_t *d_counts, int64_t cap,
                int64_t *d_n_out, int64_t *n_out_host, void *d_ws, size_t ws_bytes,
                const cga_tune *tune, cga_stream stream);

/* --------------------------------------------------------------------- kNN
 * Nearest-neighbour search, Eq. (7)-(8), generalised to k: for each of nq
 * float32 query points (AoS), quantized by the grid rule, the k voxels of the
 * CGA smallest in (squared voxel distance, key).  Outputs row-major nq x k:
 * d_idx (int64 position in the key array, -1 padding when fewer than k
 * voxels exist) and d_d2 (uint64 squared distance, UINT64_MAX padding).
 * k in [1, 32]; n (the host bound) below 2^31 (else CGA_EINVAL).  On a
 * LINEAR grid the keys are re-keyed to Morton order inside the call (a
 * key-value sort carrying each key's position; the workspace grows by about
 * 3 * (S + 4) bytes per key): d_idx then holds LINEAR positions, and ties
 * go to the smaller LINEAR position.  From 2^18 queries on, the queries
 * are searched in the order of their Morton keys (results are unchanged;
 * the workspace then grows by about 24 bytes per query, so size it with the
 * same nq as the call).  Launch knobs, read from the environment at each
 * call, change no result: CGA_KNN_ORDER (1 / 0: the Morton ordering on /
 * off), CGA_KNN_LA (level of the first round's cell, default 4),
 * CGA_KNN_QUEUE (1 / 0: teams take queries from a counter / round-robin;
 * by default the counter from 8 queries per resident team) and
 * CGA_KNN_BLOCKS (a cap on the search's grid).
 * Errors: CGA_ENONFINITE for a non-finite query (device); CGA_EMISMATCH
 * (device) when the keys are not sorted, unique and within the grid (the
 * results are then unspecified, but every access stays in bounds). */
size_t cga_knn_workspace_bytes(const cga_grid *grid, int64_t n, int64_t nq);
int cga_knn(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
            const float *d_q, int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2, void *d_ws,
            size_t ws_bytes, cga_stream stream);
/* The same search built with work counters, for measurement: identical
 * outputs, and d_work (device, 4 uint64, accumulated -- the caller zeroes
 * it) gains the search's node-record loads (16 B each), dense-table loads (4 B
 * each), voxels offered to the candidate list and walk-loop steps, summed
 * over all queries and lanes.  The search is deterministic, so these are the
 * exact per-call work of cga_knn on the same input. */
int cga_knn_count(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
                  const float *d_q, int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2,
                  uint64_t *d_work, void *d_ws, size_t ws_bytes, cga_stream stream);

/* ------------------------------------------------------------- values
 * The Value array (Section V): per-voxel attributes from per-point ones.
 * d_attr holds n packed values, four 8-bit channels each (channel c in bits
 * 8c .. 8c + 7; RGB as in Table II fits).  d_keys is the CGA of the same
 * points on the same grid (cga_build): u sorted unique keys, device count
 * d_u nullable.  d_values (u uint32) receives each voxel's channel-wise
 * average of its points' values, rounded half up, floor((2 sum + count) /
 * (2 count)) -- the averaging of colours in a grid box that Section III-B's
 * downsampling applies.  The points' keys and values are radix-sorted
 * together so that each voxel's points form one run, summed without atomics.
 * Workspace: cga_voxel_values_workspace_bytes(grid, n).  n below 2^30.
 * Errors: CGA_ENONFINITE (device) for a non-finite point; CGA_EMISMATCH
 * (device) when a point's voxel is not among the keys or a key has no point. */
size_t cga_voxel_values_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_voxel_values(const cga_grid *grid, const float *d_xyz, int64_t n, const uint32_t *d_attr,
                     const void *d_keys, int64_t u, const int64_t *d_u, uint32_t *d_values,
                     void *d_ws, size_t ws_bytes, cga_stream stream);

/* Values of a merge, Eq. (1): for every key of the union d_keys_m (cga_merge
 * of the same two CGAs), the value of the input holding it; a key in both
 * takes a's value (CGA_VALUES_BASE, a is the base cloud) or the channel-wise
 * average of the two values, rounded half up (CGA_VALUES_AVERAGE) -- the two
 * rules Section II-A gives for overlapping points.  Device counts nullable.
 * Errors: CGA_EINVAL for another policy; CGA_EMISMATCH (device) when a union
 * key is in neither input. */
enum { CGA_VALUES_BASE = 0, CGA_VALUES_AVERAGE = 1 };
size_t cga_merge_values_workspace_bytes(void);
int cga_merge_values(const cga_grid *grid, const void *d_keys_a, const uint32_t *d_values_a,
                     int64_t na, const int64_t *d_na, const void *d_keys_b,
                     const uint32_t *d_values_b, int64_t nb, const int64_t *d_nb,
                     const void *d_keys_m, int64_t nm, const int64_t *d_nm, int policy,
                     uint32_t *d_values_m, void *d_ws, size_t ws_bytes, cga_stream stream);

/* -------------------------------------------------------------- occupancy
 * Octree occupancy codes (Section II-E: constructing the octree, coding of
 * the occupancy codes) of a sorted unique MORTON key array.  The octree's
 * level-L cells are the distinct key >> 3L; a cell's code has bit o set when
 * its child in octant o (o = x_bit << 2 | y_bit << 1 | z_bit) is occupied.
 * d_occ (nullable) receives the codes of levels depth .. 1, root first, one
 * level after another, cells of a level in key order: sum_{L>=1} count[L]
 * bytes.  d_counts (nullable, depth + 1 int64) receives count[L], the
 * occupied cells per level (count[0] = n, count[depth] = 1 when n > 0).
 * n below 2^31.  Errors: CGA_ECAPACITY (device) when the codes exceed occ_cap
 * bytes (codes past occ_cap are not written); CGA_EMISMATCH (device) when the
 * keys are not sorted, unique and within the grid; CGA_EUNSUPPORTED for a
 * LINEAR grid. */
size_t cga_occupancy_workspace_bytes(const cga_grid *grid, int64_t n);
int cga_occupancy(const cga_grid *grid, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint8_t *d_occ, int64_t occ_cap, int64_t *d_counts, void *d_ws,
                  size_t ws_bytes, cga_stream stream);

/* ----------------------------------------------------------------- lookup
 * Point location and range start over a sorted unique uint64 key array (the
 * lookup of Section V-A; Table III): rank = number of keys < q (lower bound),
 * found = (rank < n && keys[rank] == q).  Plain branch-free binary search;
 * the exact baseline that the learned index below is checked against.  d_found nullable. */
int cga_binary_lookup(const uint64_t *d_keys, int64_t n, const int64_t *d_n,
                      const uint64_t *d_q, int64_t nq, int64_t *d_rank, uint8_t *d_found,
                      cga_stream stream);

/* ---------------------------------------------------------- learned index
 * A learned index over one sorted unique uint64 key array (point location
 * and range start, the lookups that dominate CGA-based compression, Table
 * III), whose results are always exactly those of cga_binary_lookup.
 *
 * Model (two stages, fitted to the array's own key -> rank function):
 *  root:  x = fl64(key - kmin) * inv_span (clamped to the key range) and
 *         leaf = clamp(floor(y(x)), 0, n_leaves - 1) with y monotone, so
 *         that leaf j owns a contiguous rank range [first_j, first_j + n_j);
 *         the root computes in fp64 (a float input would send every key of
 *         one 2^-24 step of the key range, a whole dense cluster, to one leaf).
 *         root_segments = 0: y = fma(a, x, b), a > 0, with a, b by least
 *         squares of rank * n_leaves / n on x.
 *         root_segments = R > 0: y is the piecewise-linear interpolant of
 *         (x, rank * n_leaves / n) through the keys at the R + 1 rank
 *         quantiles, clamped inside each segment (monotone by construction);
 *         the segment is found by binary search over the R + 1 knot inputs.
 *  leaf:  x_j = fl32(key - key_first_j) * inv_span_j, prediction
 *         p = clamp(first_j + rintf(n_j * f_j(x_j)), first_j, first_j + n_j)
 *         with f_j linear (least squares, fp64 sums) or a 1-16-1 ReLU network
 *         f(x) = sum_h w2_h relu(w1_h x + b1_h) + b2 (49 float32 parameters),
 *         initialised to the piecewise-linear interpolant of the leaf's
 *         rank function at its 16 rank quantiles and then trained by
 *         full-batch Adam on mean squared error for `epochs` epochs (a leaf
 *         of more than 512 keys trains on 512 of them evenly spaced by rank).
 *  window: err_lo_j / err_hi_j = min / max of (rank - p) over the leaf's keys.
 * Lookup: route, predict, take [lo, hi] = p + [err_lo, err_hi] clamped to
 * the leaf [f, f + n_j], and accept it iff (lo == 0 || keys[lo-1] < q) &&
 * (hi == n || keys[hi] >= q): one lower-bound search over [lo - 1, hi + 1)
 * decides both and finds the rank.  A failed check (an absent key the window
 * does not cover, or a key array other than the trained one) falls back to a
 * full binary search, counted in d_fallbacks.  Ranks are therefore exact for
 * any sorted key array of n keys, whatever the index holds.
 * The index is one caller-owned, position-independent device buffer of
 * cga_index_bytes (it includes a 32 KiB fingerprint).  It records n, kmin,
 * kmax and the keys at min(n, 4096) evenly spaced ranks (s * (n - 1) /
 * (m - 1) for s < m).  A lookup whose array differs in n, kmin or kmax
 * writes rank 0 / found 0 and reports CGA_EMISMATCH; one that differs at a
 * sampled rank reports CGA_EMISMATCH with exact ranks; a difference at
 * other ranks only goes undetected (the ranks stay exact). */
typedef struct {
    uint32_t n_leaves;      /* 1 .. 2^24 (4096 .. 2^20 typical) */
    uint32_t leaf_kind;     /* 0 = linear, 1 = 1-16-1 ReLU network */
    uint32_t epochs;        /* network leaves: Adam epochs (0 = keep the initialisation) */
    float lr;               /* network leaves: Adam step size */
    uint32_t root_segments; /* 0 = one linear root model; else 1 .. 65536 segments */
} cga_index_params;

size_t cga_index_bytes(const cga_index_params *params);
size_t cga_index_train_workspace_bytes(const cga_index_params *params, int64_t n);
int cga_index_train(const uint64_t *d_keys, int64_t n, const cga_index_params *params,
                    void *d_index, size_t index_bytes, void *d_ws, size_t ws_bytes,
                    cga_stream stream);
/* d_rank: int64 lower bound per query; d_found (nullable): uint8 membership;
 * d_fallbacks (nullable): uint64 counter, incremented per fallback (the
 * caller zeroes it).  d_ws: at least cga_index_lookup_workspace_bytes. */
size_t cga_index_lookup_workspace_bytes(void);
int cga_index_lookup(const void *d_index, const uint64_t *d_keys, int64_t n, const uint64_t *d_q,
                     int64_t nq, int64_t *d_rank, uint8_t *d_found, uint64_t *d_fallbacks,
                     void *d_ws, size_t ws_bytes, cga_stream stream);
/* Per-leaf window widths (err_hi - err_lo + 1, int32, n_leaves entries) and
 * key counts (int64) of a trained index, for reporting. */
int cga_index_stats(const void *d_index, int32_t *d_width, int64_t *d_count, cga_stream stream);
/* Full-batch loss and gradient of one 1-16-1 ReLU leaf network on n samples
 * (x, t), computed by the same device code the training uses: d_params (49
 * float32: w1[16], b1[16], w2[16], b2), d_grad (49 float64), d_loss (1
 * float64).  Mean squared error, (1/n) sum (f(x_i) - t_i)^2.  x must ascend
 * (as a leaf's samples do): the gradient is formed from prefix sums over each
 * hidden unit's active run, and x that does not ascend makes every output
 * NaN.  Exposed so the gradients can be checked against an independent fp64
 * computation. */
int cga_mlp_loss_grad(const float *d_params, const float *d_x, const float *d_t, int64_t n,
                      double *d_grad, double *d_loss, cga_stream stream);

/* ---------------------------------------------------------------- batched
 * CGA construction of nframes frames plus the union of every consecutive
 * pair (frame f u frame f+1, Eq. (1)), all on one grid.  d_xyz holds the
 * frames' points back to back (n in total); d_off (device, nframes + 1
 * int64) the frame boundaries, d_off[0] = 0, d_off[nframes] = n.
 * Outputs:
 *   d_keys (capacity n): each frame's sorted unique keys, frame after frame;
 *   d_counts (nullable, capacity n): points per voxel, aligned to d_keys;
 *   d_key_off (nframes + 1 int64): frame f's keys are
 *       d_keys[d_key_off[f] .. d_key_off[f+1]);
 *   d_merged (capacity 2n): pair f's union starts at d_merged_off[f]
 *       (nframes - 1 int64) and holds d_merged_cnt[f] keys.
 * Implementation: composite keys (frame << 3*depth | key), a radix sort
 * segmented by frame (each frame's keys sorted within the frame's range by
 * the 3*depth key bits alone; above 4096 frames one sort of the composite
 * keys, frame bits included), one run-length pass, per-frame offsets by
 * binary search, then one persistent merge launch over a window queue
 * spanning all pairs.  Every size
 * after the input stays on the device, so the call can be captured in a
 * graph: cga_batch_graph_create records it once (on a private stream) into
 * an executable graph that cga_batch_graph_launch replays on any stream,
 * with the same buffers.  Requires 3 * depth + ceil(log2(nframes)) <= 64;
 * nframes in [1, 65536]; n < 2^30.  tune NULL = autotuned (see below) or
 * default digit width and tile size; results never depend on it. */
size_t cga_batch_workspace_bytes(const cga_grid *grid, int nframes, int64_t n);
/* Key bits the batched sort's passes cover for nframes frames on this grid
 * (3*depth when segmented, else 3*depth + ceil(log2(nframes))): the
 * key_bits under which cga_autotune_sort records a choice that
 * cga_batch_build_merge and cga_batch_graph_create then use.  0 when the grid
 * or nframes is invalid. */
int cga_batch_sort_bits(const cga_grid *grid, int nframes);
int cga_batch_build_merge(const cga_grid *grid, const float *d_xyz, const int64_t *d_off,
                          int nframes, int64_t n, void *d_keys, uint32_t *d_counts,
                          int64_t *d_key_off, void *d_merged, int64_t *d_merged_off,
                          int64_t *d_merged_cnt, const cga_tune *tune, void *d_ws,
                          size_t ws_bytes, cga_stream stream);
int cga_batch_graph_create(const cga_grid *grid, const float *d_xyz, const int64_t *d_off,
                           int nframes, int64_t n, void *d_keys, uint32_t *d_counts,
                           int64_t *d_key_off, void *d_merged, int64_t *d_merged_off,
                           int64_t *d_merged_cnt, const cga_tune *tune, void *d_ws,
                           size_t ws_bytes, void **graph);
int cga_batch_graph_launch(void *graph, cga_stream stream);
int cga_batch_graph_destroy(void *graph);

/* -------------------------------------------------------------- autotuner
 * Times every compiled (radix_bits, tile_items) pair of the radix sort on n
 * keys of key_bytes width and key_bits significant bits -- a copy of d_keys,
 * or synthetic hashed keys when d_keys is NULL -- and records the fastest for
 * (key_bytes, key_bits, floor(log2 n)).  Later calls with tune == NULL
 * (build, project, batched) use a recorded choice when one matches.  When
 * the environment variable CGA_TUNE_CACHE names a file, recorded choices are
 * loaded from it on first use and appended to it.  Returns the choice and its
 * best time in milliseconds. */
size_t cga_autotune_workspace_bytes(uint32_t key_bytes, int64_t n);
int cga_autotune_sort(const void *d_keys, uint32_t key_bytes, uint32_t key_bits, int64_t n,
                      void *d_ws, size_t ws_bytes, cga_tune *best, float *best_ms,
                      cga_stream stream);

/* ---------------------------------------------------------------- timing
 * Per-kernel launch timing for measurement.  After cga_prof_enable, each
 * launch of a kernel whose label is in the comma-separated `filter` (NULL or
 * "" = every kernel) is bracketed by two HIP events on the launch's own
 * stream.  cga_prof_read waits for all pending events and returns the summed
 * duration and launch count of one label since the last reset.  Labels:
 * begin, encode, histogram, hist_scan, onesweep, rle, arrays,
 * merge_partition, merge, rekey, knn, binary_lookup.  Not for graph capture. */
int cga_prof_enable(const char *filter);
int cga_prof_disable(void);
int cga_prof_reset(void);
int cga_prof_read(const char *label, double *total_ms, int64_t *launches);
/* Attainable HBM bandwidth probe (the roofline's measured ceiling beside the
 * datasheet peak): mode 0 copies `bytes` from d_src to d_dst (each byte read
 * once and written once), mode 1 only reads d_src (d_dst nullable: a 4-byte
 * sink that is never written in practice).  bytes a positive multiple of 16;
 * `blocks` workgroups of 256 threads, grid-stride. */
int cga_stream_probe(const void *d_src, void *d_dst, size_t bytes, int mode, int blocks,
                     cga_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* CGA_H */
