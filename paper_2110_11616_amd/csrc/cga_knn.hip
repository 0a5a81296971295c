// k-nearest-neighbour search, Eq. (7)-(8) generalised to k, over a sorted
// unique MORTON key array, and plain binary-search point lookup.
//
// In Morton order every octree cell is a contiguous run of keys, so the array
// already is a pointer-free octree; searching it directly costs a binary
// search for every cell visited.  Each call therefore first derives the
// explicit octree of the array, level by level from the voxels up (node
// counts, a scan, node indexes, then per level the node words, and the
// oriented boxes of the lower levels from their voxels):
//   level-L node j (L = 1..depth) is the j-th distinct prefix key >> 3L;
//   its first 64-bit word holds first and mask, where first indexes its
//   first child at level L - 1 (a key index at L = 1) and bit o of mask says
//   whether the child in octant o exists, plus the axis-aligned box of its
//   voxels; its second word an oriented box of its voxels (a slab along
//   their least-variance direction).  Child o is node first + popcount(mask
//   below bit o): one 16-byte load per visited node, and no load at all for
//   the voxels under a level-1 node, whose coordinates follow from the path.
//   The boxes bound the distance from a query to a node's voxels: a child
//   whose axis-aligned box, cut to its parent's, lies beyond the k-th
//   distance is never loaded, and a loaded node whose oriented box does
//   opens no child.
// A dense table maps every level-DT cell (DT = depth - DL, 8^DL cells, DL up
// to 7 and no more than about log8 of the key count, so that clearing it
// costs no more than the keys themselves) to its node, so a search enters the
// tree near the bottom instead of at the root.
//
// Queries: a team of 8 lanes answers one query at a time.  Round 0 searches
// the query's level-LA cell: lane t walks child t (in visiting order) of each
// of the cell's eight children, depth-first, nearest child first, pruning
// cells whose nearest point is strictly farther than the team's current k-th
// distance (so ties survive); a lane whose walks are over takes over the
// remaining children of a busy lane's shallowest open node.  The team keeps
// one candidate list, ordered by (squared distance, key index), spread over
// its lanes.  If the k-th distance ball is not inside the searched cell, the
// next round searches the up to 8 cells of the smallest level that cover the
// ball's bounding cube (their children dealt out the same way), and repeats
// with the grown ball until a round that started from a known bound covers
// it.  The teams of a wave do not wait for each other: each goes on with its
// next round or query.
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "cga_common.h"
#include "cga_sort.h"

namespace cga {

constexpr int kKnnBlock = 256;
constexpr int kCells = 8;  // start cells of a round, children of a node
// Lanes per query: 16 from k = 9 on (more work per query to share out: 1M
// queries, k = 16, over 2 x 10M sphere points at depth 14, 59.6 against
// 63.1 ms), else 8 (100k queries, k = 8, over 2 x 1M LiDAR points at depth
// 12: 0.81 against 1.04 ms with 16).
template <int KT>
constexpr int knn_team() {
    return KT >= 16 ? 16 : 8;
}
constexpr int kMaxDepth = 21;
constexpr int kTreeRows = 4;                       // rows of 256 keys per build tile
constexpr int kTreeTile = kTreeRows * 256;         // keys per build tile
constexpr int kLaDefault = 4;                      // round-0 cell level
constexpr uint32_t kPackedDepth = 15;              // deepest grid with 32-bit squared distances
// Large query sets are answered in the order of the top kOrderBits of their
// Morton keys (a 3-pass sort of index << kOrderBits | key bits), so that the
// teams of a wave search neighbouring regions: similar costs, shared nodes.
constexpr int kOrderBits = 24;
constexpr int64_t kOrderMin = (int64_t)1 << 18;

template <typename K>
__device__ __forceinline__ int64_t lower_bound_dev(const K *keys, int64_t n, K q) {
    if (n <= 0) return 0;
    int64_t lo = 0, len = n;
    while (len > 1) {
        int64_t half = len >> 1;
        lo = keys[lo + half] < q ? lo + half : lo;
        len -= half;
    }
    return lo + (keys[lo] < q ? 1 : 0);
}

// ------------------------------------------------------------ octree build
// Levels the dense table spans for n keys: floor(log8 n), within [2, 7].
inline int dense_levels(int64_t n) {
    int dl = 2;
    while (dl < 7 && ((int64_t)1 << (3 * (dl + 1))) <= n) ++dl;
    return dl;
}
__host__ __device__ inline int dense_level(uint32_t depth, int dl) {
    return (int)depth > dl ? (int)depth - dl : 0;
}
__host__ __device__ inline int64_t dense_cells(uint32_t depth, int dl) {
    return dense_level(depth, dl) > 0 ? (int64_t)1 << (3 * dl) : 0;
}

// Highest level at which key i starts a new cell: key 0 starts every cell up
// to the root (level depth); key i > 0 starts the cells of every level below
// the highest bit in which it differs from key i - 1.  -1 past the end (and
// for a repeated key, which valid input never has).
template <typename K>
__device__ __forceinline__ int head_level(const K *keys, int64_t i, int64_t n, uint32_t depth) {
    if (i >= n) return -1;
    if (i == 0) return (int)depth;
    const uint64_t x = (uint64_t)keys[i] ^ (uint64_t)keys[i - 1];
    return x ? (63 - __clzll(x)) / 3 : -1;
}

// Number of keys: the device count when given, never above the host bound.
__device__ __forceinline__ int64_t key_count(int64_t n_host, const int64_t *d_n) {
    const int64_t n = dev_count(n_host, d_n);
    return n < n_host ? n : n_host;
}

// The level table: lvl[L] = nodes at level L (lvl[0] = keys), lvl[kLvlBase +
// L] = first node of level L in the concatenated arrays (L = 1 .. depth + 1,
// the last being the total), and lvl[kLvlTotal] = the total, or -1 when it
// exceeds the arrays (a key array that is not a CGA of the grid can have
// more cells than the bound).
constexpr int kLvlBase = kMaxDepth + 2;
constexpr int kLvlTotal = 2 * kMaxDepth + 4;
constexpr int kLvlWords = 2 * kMaxDepth + 6;

__device__ __forceinline__ int64_t tree_total(const int64_t *lvl) { return lvl[kLvlTotal]; }

// The node bases and the total, from the level sizes (one thread).
__global__ void k_tree_bases(int64_t *__restrict__ lvl, uint32_t depth, int64_t nodes_max) {
    if (threadIdx.x != 0) return;
    int64_t b = 0;
    for (uint32_t L = 1; L <= depth; ++L) {
        lvl[kLvlBase + L] = b;
        b += lvl[L];
    }
    lvl[kLvlBase + depth + 1] = b;
    lvl[kLvlTotal] = b <= nodes_max ? b : -1;
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Pass 1: per tile of kTreeTile keys, the number of nodes each level starts
// in it (cnt[(L - 1) * tiles + tile]); also clears the dense entry table.
template <typename K>
__global__ __launch_bounds__(256) void k_tree_count(const K *__restrict__ keys, int64_t n_host,
                                                    const int64_t *d_n, uint32_t depth,
                                                    int64_t tiles, uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ dense, int64_t ncells,
                                                    uint32_t *err) {
    __shared__ uint32_t s_c[kMaxDepth + 1];
    const int64_t n = key_count(n_host, d_n);
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * 256)
        dense[c] = 0;
    if (threadIdx.x <= kMaxDepth) s_c[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int r = 0; r < kTreeRows; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kTreeTile + r * 256 + threadIdx.x;
        const int h = head_level(keys, i, n, depth);
        // not a CGA of this grid: unsorted, repeated, or wider than 3 * depth bits
        if (i < n && ((i > 0 && keys[i] <= keys[i - 1]) || ((uint64_t)keys[i] >> (3 * depth)) != 0))
            set_err(err, ERR_MISMATCH);
        for (uint32_t L = 1; L <= depth; ++L) {
            const uint64_t b = __ballot(h >= (int)L);
            if (!b) break;
            if (lane == 0) atomicAdd(&s_c[L], (uint32_t)__popcll(b));
        }
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= depth)
        cnt[(int64_t)(threadIdx.x - 1) * tiles + blockIdx.x] = s_c[threadIdx.x];
}

// Pass 2: one block per level; exclusive scan of the tile counts in place,
// level size into lvl[L] (lvl[0] = number of keys).
__global__ __launch_bounds__(1024) void k_tree_scan(uint32_t *__restrict__ cnt, int64_t tiles,
                                                    int64_t n_host, const int64_t *d_n,
                                                    int64_t *__restrict__ lvl) {
    __shared__ uint32_t s_w[16];
    const int L = blockIdx.x + 1;
    uint32_t *c = cnt + (int64_t)(L - 1) * tiles;
    const int64_t per = (tiles + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    const int64_t b1 = b0 + per < tiles ? b0 + per : tiles;
    uint32_t sum = 0;
    for (int64_t t = b0; t < b1; ++t) sum += c[t];
    // block exclusive scan of the per-thread sums
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < 16; ++w) {
        before += w < wave ? s_w[w] : 0;
        total += s_w[w];
    }
    uint32_t run = before + incl - sum;
    for (int64_t t = b0; t < b1; ++t) {
        const uint32_t v = c[t];
        c[t] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        lvl[L] = total;
        if (L == 1) lvl[0] = key_count(n_host, d_n);
    }
}

// Pass 3: node index of every cell each key starts, at every level; writes
// the first-child index and the octant of each node, and the dense entry of
// each level-DT node.  Level offsets: node arrays of all levels are
// concatenated, level L starting at base(L) = lvl[1] + ... + lvl[L - 1].
template <typename K>
__global__ __launch_bounds__(256) void k_tree_build(const K *__restrict__ keys, int64_t n_host,
                                                    const int64_t *d_n, uint32_t depth, int dt,
                                                    int64_t tiles, const uint32_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ lvl,
                                                    uint32_t *__restrict__ first,
                                                    uint32_t *__restrict__ kfirst,
                                                    uint8_t *__restrict__ oct,
                                                    uint32_t *__restrict__ dense, int64_t ncells,
                                                    int64_t nodes_max) {
    __shared__ uint32_t s_w[kTreeRows][4][kMaxDepth + 1];
    __shared__ int64_t s_base[kMaxDepth + 2];
    __shared__ uint32_t s_off[kMaxDepth + 1];
    __shared__ int s_max[4];
    if (tree_total(lvl) < 0) return;  // block-uniform
    const int64_t n = key_count(n_host, d_n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x >= 1 && threadIdx.x <= depth + 1) s_base[threadIdx.x] = lvl[kLvlBase + threadIdx.x];
    if (threadIdx.x >= 1 && threadIdx.x <= depth)
        s_off[threadIdx.x] = cnt[(int64_t)(threadIdx.x - 1) * tiles + blockIdx.x];
    int h[kTreeRows];
    int hmax = -1;
#pragma unroll
    for (int r = 0; r < kTreeRows; ++r) {
        h[r] = head_level(keys, (int64_t)blockIdx.x * kTreeTile + r * 256 + threadIdx.x, n, depth);
        hmax = h[r] > hmax ? h[r] : hmax;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int v = __shfl_xor(hmax, o, 64);
        hmax = v > hmax ? v : hmax;
    }
    if (lane == 0) s_max[wave] = hmax;
    __syncthreads();
    int bmax = s_max[0];
    for (int w = 1; w < 4; ++w) bmax = s_max[w] > bmax ? s_max[w] : bmax;
    // wave counts of the nodes each level starts, per row
#pragma unroll
    for (int r = 0; r < kTreeRows; ++r)
        for (int L = 1; L <= bmax; ++L) {
            const uint64_t b = __ballot(h[r] >= L);
            if (lane == 0) s_w[r][wave][L] = (uint32_t)__popcll(b);
        }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTreeRows; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kTreeTile + r * 256 + threadIdx.x;
        int64_t child = i;  // this key's node one level down (the key itself at level 0)
        for (int L = 1; L <= bmax; ++L) {
            const uint64_t b = __ballot(h[r] >= L);
            if (!b) break;
            uint32_t before = s_off[L];
            for (int rr = 0; rr < r; ++rr)
                for (int w = 0; w < 4; ++w) before += s_w[rr][w][L];
            for (int w = 0; w < wave; ++w) before += s_w[r][w][L];
            if (h[r] >= L) {
                const int64_t j = (int64_t)before + mbcnt64(b);
                const int64_t t = s_base[L] + j;
                first[t] = (uint32_t)child;
                kfirst[t] = (uint32_t)i;
                oct[t] = (uint8_t)(((uint64_t)keys[i] >> (3 * L)) & 7);
                const uint64_t dc = (uint64_t)keys[i] >> (3 * dt);
                if (L == dt && dc < (uint64_t)ncells) dense[dc] = (uint32_t)j + 1;
                child = j;
            }
        }
    }
}

// Node word: child mask in bits 0-7, first child index in bits 8-38, and in
// bits 40-63 the bounding box of the node's voxels, per axis a (x, y, z) a
// 4-bit low and high bound at bits 40 + 8a and 44 + 8a, in units of 1/16 of
// the cell (of a voxel below level 4): voxel offsets [lo << s, ((hi + 1) << s)
// - 1] within the cell, s = max(level - 4, 0), rounded outwards.  On a
// surface a cell's voxels fill a thin slab of it, so distances to the box
// bound the distances to the voxels far more tightly than the cell's do.
constexpr uint64_t kNodeFirstMask = 0x7FFFFFFFull;
constexpr int kScanLevels = 6;  // levels whose oriented boxes are fitted to the voxels
constexpr int kTreeBigCtr = 24;  // control-block counters of the big-node lists, one per level
constexpr int kLinearSortCtr = 8;  // tile counters of the LINEAR keys' re-key sort (up to 8 passes)
constexpr int kKnnQueryCtr = 20;   // control-block counter of the search's query queue
constexpr int kObbMinLevel = 8;    // least start-cell level of a round that tests oriented boxes
constexpr int64_t kKnnQueuePerTeam = 8;  // queries per team from which the search uses it
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
constexpr int kNodeBoxShift = 40;
__host__ __device__ __forceinline__ int64_t node_first(uint64_t w) {
    return (int64_t)((w >> 8) & kNodeFirstMask);
}
__device__ __forceinline__ int box_unit_shift(int level) { return level > 4 ? level - 4 : 0; }
__device__ __forceinline__ void node_box(uint64_t w, int a, int level, uint32_t &lo, uint32_t &hi) {
    const int s = box_unit_shift(level);
    const uint32_t f = (uint32_t)(w >> (kNodeBoxShift + 8 * a));
    lo = (f & 15u) << s;
    hi = ((((f >> 4) & 15u) + 1u) << s) - 1u;
}

// Second word of a node: an oriented box holding the node's voxels.  Its
// axes are n, the direction in which the voxel positions vary least (on a
// surface, its normal), stored octahedrally in 7 + 7 bits, and e1, e2, which
// complete the decoded n to an orthonormal frame; per axis an 8-bit signed
// range [lo, hi] of the voxels' offsets from the cell centre along it, in
// units of 1/128 of the cell, rounded outwards.  A far query sees a surface
// cell's voxels in a slab a few voxels thick along n, while its axis-aligned
// box can be as deep as the cell: the distance to the oriented box bounds the
// distance to the voxels far more tightly.  (Bits: u 0-6, v 7-13, then lo,
// hi of n at 14 and 22, of e1 at 30 and 38, of e2 at 46 and 54.)
struct Frame {
    float a[3][3];  // rows n, e1, e2
};

__device__ __forceinline__ float sgnf(float v) { return v >= 0.f ? 1.f : -1.f; }

__device__ __forceinline__ uint32_t oct_encode(float x, float y, float z) {
    float l1 = fabsf(x) + fabsf(y) + fabsf(z);
    if (!(l1 > 0.f)) {
        x = 0.f;
        y = 0.f;
        z = 1.f;
        l1 = 1.f;
    }
    float px = x / l1, py = y / l1;
    if (z < 0.f) {
        const float tx = (1.f - fabsf(py)) * sgnf(px), ty = (1.f - fabsf(px)) * sgnf(py);
        px = tx;
        py = ty;
    }
    const int u = min(max((int)rintf((px * 0.5f + 0.5f) * 127.f), 0), 127);
    const int v = min(max((int)rintf((py * 0.5f + 0.5f) * 127.f), 0), 127);
    return (uint32_t)u | ((uint32_t)v << 7);
}

__device__ __forceinline__ Frame frame_decode(uint32_t code) {
    float px = (float)(code & 127u) * (2.f / 127.f) - 1.f;
    float py = (float)((code >> 7) & 127u) * (2.f / 127.f) - 1.f;
    const float pz = 1.f - fabsf(px) - fabsf(py);
    if (pz < 0.f) {
        const float tx = (1.f - fabsf(py)) * sgnf(px), ty = (1.f - fabsf(px)) * sgnf(py);
        px = tx;
        py = ty;
    }
    Frame f;
    const float r = rsqrtf(px * px + py * py + pz * pz);
    const float n0 = px * r, n1 = py * r, n2 = pz * r;
    // e1 = n x (the unit axis along which n is smallest), normalised
    const float ax = fabsf(n0), ay = fabsf(n1), az = fabsf(n2);
    float c0, c1, c2;
    if (ax <= ay && ax <= az) {  // axis x
        c0 = 0.f;
        c1 = n2;
        c2 = -n1;
    } else if (ay <= az) {  // axis y
        c0 = -n2;
        c1 = 0.f;
        c2 = n0;
    } else {  // axis z
        c0 = n1;
        c1 = -n0;
        c2 = 0.f;
    }
    const float rc = rsqrtf(c0 * c0 + c1 * c1 + c2 * c2);
    c0 *= rc;
    c1 *= rc;
    c2 *= rc;
    f.a[0][0] = n0;
    f.a[0][1] = n1;
    f.a[0][2] = n2;
    f.a[1][0] = c0;
    f.a[1][1] = c1;
    f.a[1][2] = c2;
    f.a[2][0] = n1 * c2 - n2 * c1;
    f.a[2][1] = n2 * c0 - n0 * c2;
    f.a[2][2] = n0 * c1 - n1 * c0;
    return f;
}

__device__ __forceinline__ int obb_lo(uint64_t w, int k) { return (int)(int8_t)(uint8_t)(w >> (14 + 16 * k)); }
__device__ __forceinline__ int obb_hi(uint64_t w, int k) { return (int)(int8_t)(uint8_t)(w >> (22 + 16 * k)); }

// Squared distance from the offset dq (query minus the centre of a level-l
// cell) to the cell's oriented box w, less safety margins that cover the
// rounding of the projections and of the frame, so that it never exceeds
// the squared distance to any voxel of the cell.
__device__ __forceinline__ float obb_dist2(uint64_t w, int l, float dq0, float dq1, float dq2) {
    const Frame f = frame_decode((uint32_t)w & 0x3FFFu);
    const float cell = (float)(1u << l), u = cell * (1.f / 128.f);
    const float margin = (fabsf(dq0) + fabsf(dq1) + fabsf(dq2)) * (1.f / 262144.f) + cell * (1.f / 1024.f);
    float d2 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float t = f.a[k][0] * dq0 + f.a[k][1] * dq1 + f.a[k][2] * dq2;
        const float lo = (float)obb_lo(w, k) * u, hi = (float)obb_hi(w, k) * u;
        const float g = fmaxf(fmaxf(lo - t, t - hi), 0.f) - margin;
        d2 += g > 0.f ? g * g : 0.f;
    }
    return d2 * (1.f - 1.f / 65536.f);
}

// Pass 4, one launch per level from the voxels up (a level's boxes are the
// union of its children's): one thread per node of level lev, the child mask
// from the children's octants, the box, and the packed node word.  With emit
// set, the masks are also the octree's occupancy codes, written to occ
// (nullable) root first, level by level, cells in key order (level L starts
// after the codes of levels depth .. L + 1), and counts (nullable) gets the
// cells per level.
template <typename K>
__global__ __launch_bounds__(256) void k_tree_mask(const K *__restrict__ keys, uint32_t depth,
                                                   uint32_t lev, const int64_t *__restrict__ lvl,
                                                   const uint32_t *__restrict__ first,
                                                   const uint8_t *__restrict__ oct,
                                                   uint64_t *__restrict__ node, float *__restrict__ mom,
                                                   int64_t nodes_max, bool emit,
                                                   uint8_t *__restrict__ occ,
                                                   int64_t occ_cap, int64_t *__restrict__ counts,
                                                   uint32_t *err) {
    __shared__ int64_t s_n[kMaxDepth + 2], s_base[kMaxDepth + 2];
    if (threadIdx.x <= depth + 1) {
        s_n[threadIdx.x] = lvl[threadIdx.x];
        s_base[threadIdx.x] = lvl[kLvlBase + threadIdx.x];
    }
    __syncthreads();
    const int64_t total = tree_total(lvl) > 0 ? tree_total(lvl) : 0;  // 0: nothing to do
    if (emit && lev == 1 && blockIdx.x == 0) {
        if (counts && threadIdx.x <= depth) counts[threadIdx.x] = s_n[threadIdx.x];
        if (threadIdx.x == 0 && occ && total > occ_cap) set_err(err, ERR_CAPACITY);
    }
    if (total == 0) return;  // block-uniform: no keys, or an oversized tree
    const uint32_t L = lev;
    const int ps = box_unit_shift((int)L);
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < s_n[L]; j += (int64_t)gridDim.x * 256) {
        const int64_t t = s_base[L] + j;
        const int64_t f0 = first[t];
        int64_t f1 = j + 1 < s_n[L] ? (int64_t)first[t + 1] : s_n[L - 1];
        if (f1 > f0 + 8) f1 = f0 + 8;  // eight children at most (unique keys)
        uint32_t mask = 0;
        uint32_t lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0u, 0u, 0u};
        // moments of the voxel offsets from this cell's centre: count, sums,
        // and the sums of products xx, yy, zz, xy, xz, yz
        float mc = 0.f, ms[3] = {0.f, 0.f, 0.f}, mS[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const float half = (float)(1u << L) * 0.5f;  // child centre = cell centre + off - 2^(L-2)
        for (int64_t c = f0; c < f1; ++c) {
            const uint32_t o = L == 1 ? (uint32_t)((uint64_t)keys[c] & 7) : oct[s_base[L - 1] + c];
            mask |= 1u << o;
            const uint64_t cw = L == 1 ? 0ull : node[2 * (s_base[L - 1] + c)];
            float dl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // the child's cell sits at offset bit(o, a) * 2^(L - 1) of this cell
                const uint32_t off = ((o >> (2 - a)) & 1u) << (L - 1);
                uint32_t clo = 0, chi = 0;
                if (L > 1) node_box(cw, a, (int)L - 1, clo, chi);
                lo[a] = min(lo[a], off + clo);
                hi[a] = max(hi[a], off + chi);
                dl[a] = (float)off - half * 0.5f;  // child centre minus this centre (voxel: -0.5 or 0.5)
            }
            if (L == 1) {
                mc += 1.f;
                ms[0] += dl[0];
                ms[1] += dl[1];
                ms[2] += dl[2];
                mS[0] += dl[0] * dl[0];
                mS[1] += dl[1] * dl[1];
                mS[2] += dl[2] * dl[2];
                mS[3] += dl[0] * dl[1];
                mS[4] += dl[0] * dl[2];
                mS[5] += dl[1] * dl[2];
            } else {
                const float *cm = mom + 10 * (s_base[L - 1] + c);
                const float m = cm[0], s0 = cm[1], s1 = cm[2], s2 = cm[3];
                mc += m;
                ms[0] += s0 + m * dl[0];
                ms[1] += s1 + m * dl[1];
                ms[2] += s2 + m * dl[2];
                mS[0] += cm[4] + 2.f * dl[0] * s0 + m * dl[0] * dl[0];
                mS[1] += cm[5] + 2.f * dl[1] * s1 + m * dl[1] * dl[1];
                mS[2] += cm[6] + 2.f * dl[2] * s2 + m * dl[2] * dl[2];
                mS[3] += cm[7] + dl[0] * s1 + dl[1] * s0 + m * dl[0] * dl[1];
                mS[4] += cm[8] + dl[0] * s2 + dl[2] * s0 + m * dl[0] * dl[2];
                mS[5] += cm[9] + dl[1] * s2 + dl[2] * s1 + m * dl[1] * dl[2];
            }
        }
        uint64_t box = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            box |= (uint64_t)(((lo[a] >> ps) & 15u) | (((hi[a] >> ps) & 15u) << 4)) << (8 * a);
        float *pm = mom + 10 * t;
        pm[0] = mc;
        pm[1] = ms[0];
        pm[2] = ms[1];
        pm[3] = ms[2];
#pragma unroll
        for (int e = 0; e < 6; ++e) pm[4 + e] = mS[e];
        // least-variance direction: power iteration on tr(C) I - C, whose
        // largest eigenvalue belongs to C's smallest
        const float inv = 1.f / mc;
        const float mu0 = ms[0] * inv, mu1 = ms[1] * inv, mu2 = ms[2] * inv;
        const float cxx = mS[0] * inv - mu0 * mu0, cyy = mS[1] * inv - mu1 * mu1, czz = mS[2] * inv - mu2 * mu2;
        const float cxy = mS[3] * inv - mu0 * mu1, cxz = mS[4] * inv - mu0 * mu2, cyz = mS[5] * inv - mu1 * mu2;
        const float tr = cxx + cyy + czz;
        float v0 = cxx <= cyy && cxx <= czz ? 1.f : 0.3f, v1 = cyy < cxx && cyy <= czz ? 1.f : 0.3f,
              v2 = czz < cxx && czz < cyy ? 1.f : 0.3f;
        for (int it = 0; it < 12; ++it) {
            const float w0 = (tr - cxx) * v0 - cxy * v1 - cxz * v2;
            const float w1 = -cxy * v0 + (tr - cyy) * v1 - cyz * v2;
            const float w2 = -cxz * v0 - cyz * v1 + (tr - czz) * v2;
            const float nn = w0 * w0 + w1 * w1 + w2 * w2;
            if (!(nn > 1e-30f)) break;
            const float r = rsqrtf(nn);
            v0 = w0 * r;
            v1 = w1 * r;
            v2 = w2 * r;
        }
        const uint32_t code = oct_encode(v0, v1, v2);
        const Frame f = frame_decode(code);
        // ranges along the frame: at level 1 from the voxels (the
        // children), at levels 2 .. kScanLevels from the voxels by
        // k_tree_ranges, above from the corners of the children's boxes
        const bool own = L == 1 || L > (uint32_t)kScanLevels;
        float tmin[3] = {3e38f, 3e38f, 3e38f}, tmax[3] = {-3e38f, -3e38f, -3e38f};
        for (int64_t c = own ? f0 : f1; c < f1; ++c) {
            const uint32_t o = L == 1 ? (uint32_t)((uint64_t)keys[c] & 7) : oct[s_base[L - 1] + c];
            float dl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) dl[a] = (float)(((o >> (2 - a)) & 1u) << (L - 1)) - half * 0.5f;
            if (L == 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float tt = f.a[k][0] * dl[0] + f.a[k][1] * dl[1] + f.a[k][2] * dl[2];
                    tmin[k] = fminf(tmin[k], tt);
                    tmax[k] = fmaxf(tmax[k], tt);
                }
            } else {
                const uint64_t cw2 = node[2 * (s_base[L - 1] + c) + 1];
                const Frame fc = frame_decode((uint32_t)cw2 & 0x3FFFu);
                const float uc = (float)(1u << (L - 1)) * (1.f / 128.f);
                float r0[3], r1[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    r0[k] = (float)obb_lo(cw2, k) * uc;
                    r1[k] = (float)obb_hi(cw2, k) * uc;
                }
#pragma unroll
                for (int corner = 0; corner < 8; ++corner) {
                    const float t0 = (corner & 1) ? r1[0] : r0[0], t1 = (corner & 2) ? r1[1] : r0[1],
                                t2 = (corner & 4) ? r1[2] : r0[2];
                    float pc[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) pc[a] = dl[a] + t0 * fc.a[0][a] + t1 * fc.a[1][a] + t2 * fc.a[2][a];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float tt = f.a[k][0] * pc[0] + f.a[k][1] * pc[1] + f.a[k][2] * pc[2];
                        tmin[k] = fminf(tmin[k], tt);
                        tmax[k] = fmaxf(tmax[k], tt);
                    }
                }
            }
        }
        uint64_t ob = code;
        if (own) {
            const float cell = (float)(1u << L), u = cell * (1.f / 128.f), slack = cell * (1.f / 1024.f);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                // never wider than the cell's own extent along the axis
                const float sup = (fabsf(f.a[k][0]) + fabsf(f.a[k][1]) + fabsf(f.a[k][2])) * (cell - 1.f) * 0.5f;
                const float a0 = fmaxf(tmin[k], -sup) - slack, a1 = fminf(tmax[k], sup) + slack;
                const int q0 = max((int)floorf(a0 / u), -128), q1 = min((int)ceilf(a1 / u), 127);
                ob |= (uint64_t)(uint8_t)(int8_t)q0 << (14 + 16 * k);
                ob |= (uint64_t)(uint8_t)(int8_t)q1 << (22 + 16 * k);
            }
        }
        node[2 * t] = (box << kNodeBoxShift) | ((uint64_t)f0 << 8) | mask;
        node[2 * t + 1] = ob;
        if (emit && occ) {
            const int64_t o = total - s_base[L + 1] + j;  // codes of levels above L come first
            if (o < occ_cap) occ[o] = (uint8_t)mask;
        }
    }
}

// Pass 5 for levels 2 .. kScanLevels, after pass 4 of the level: the
// oriented box's ranges from the node's own voxels (its keys
// [kfirst[t], kfirst[t + 1]) of the level, decoded), so that they are as
// tight as the voxels allow.  Above kScanLevels the children hold enough
// voxels for well-defined normals, and their box corners bound the parent's
// ranges closely enough.
//
// Voxel offsets of keys [k0, k1) from the cell centre (cx, cy, cz),
// projected on the frame's axes: their least and greatest, over the keys
// i = k0 + sub, k0 + sub + step, ... (four loads in flight per round: a big
// node's scan is bound by load latency, not by the projections).
template <typename K>
__device__ __forceinline__ void frame_extent(const K *__restrict__ keys, int64_t k0, int64_t k1,
                                             int sub, int step, uint32_t depth, const Frame &f,
                                             float cx, float cy, float cz, float tmin[3],
                                             float tmax[3]) {
    constexpr int kIn = 4;
    for (int64_t i0 = k0 + sub; i0 < k1; i0 += (int64_t)step * kIn) {
        K kk[kIn];
#pragma unroll
        for (int m = 0; m < kIn; ++m) {
            const int64_t i = i0 + (int64_t)m * step;
            kk[m] = keys[i < k1 ? i : k0];  // repeating the first key changes no range
        }
#pragma unroll
        for (int m = 0; m < kIn; ++m) {
            const Vox v = dec3((uint64_t)kk[m], depth, false);
            const float d0 = (float)v.x - cx, d1 = (float)v.y - cy, d2 = (float)v.z - cz;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float tt = f.a[k][0] * d0 + f.a[k][1] * d1 + f.a[k][2] * d2;
                tmin[k] = fminf(tmin[k], tt);
                tmax[k] = fmaxf(tmax[k], tt);
            }
        }
    }
}

// Two launches per level: BIG = false, a thread per node, which fits the
// nodes of at most kSmallNode keys and lists the others (big, *n_big); BIG
// = true, a wave per listed node (its lanes stride over the keys).  Sparse
// levels (a few voxels per cell) and dense ones (a LiDAR ground plane) both
// keep their lanes busy.
constexpr int64_t kSmallNode = 16;

template <typename K, bool BIG>
__global__ __launch_bounds__(256) void k_tree_ranges(const K *__restrict__ keys, uint32_t depth,
                                                     uint32_t lev, const int64_t *__restrict__ lvl,
                                                     const uint32_t *__restrict__ kfirst,
                                                     uint64_t *__restrict__ node,
                                                     uint32_t *__restrict__ big, uint32_t *n_big) {
    constexpr int LANES = BIG ? 64 : 1;
    __shared__ int64_t s_n[kMaxDepth + 2], s_base[kMaxDepth + 2];
    if (threadIdx.x <= depth + 1) {
        s_n[threadIdx.x] = lvl[threadIdx.x];
        s_base[threadIdx.x] = lvl[kLvlBase + threadIdx.x];
    }
    __syncthreads();
    if (tree_total(lvl) <= 0) return;  // block-uniform: no keys, or an oversized tree
    const uint32_t L = lev;
    const int sub = (int)(threadIdx.x % LANES);
    const int64_t per_block = 256 / LANES;
    const float cell = (float)(1u << L), u = cell * (1.f / 128.f), slack = cell * (1.f / 1024.f);
    const float hc = (cell - 1.f) * 0.5f;
    const int64_t nl = BIG ? (int64_t)ld_agent(n_big) : s_n[L];
    for (int64_t q = (int64_t)blockIdx.x * per_block + threadIdx.x / LANES; q < nl;
         q += (int64_t)gridDim.x * per_block) {
        const int64_t j = BIG ? (int64_t)big[q] : q;
        const int64_t t = s_base[L] + j;
        const int64_t k0 = kfirst[t], k1 = j + 1 < s_n[L] ? (int64_t)kfirst[t + 1] : s_n[0];
        if (!BIG && k1 - k0 > kSmallNode) {
            big[atomicAdd(n_big, 1u)] = (uint32_t)j;
            continue;
        }
        const uint64_t w1 = node[2 * t + 1];
        const Frame f = frame_decode((uint32_t)w1 & 0x3FFFu);
        const Vox v0 = dec3((uint64_t)keys[k0], depth, false);
        float tmin[3] = {3e38f, 3e38f, 3e38f}, tmax[3] = {-3e38f, -3e38f, -3e38f};
        frame_extent(keys, k0, k1, sub, LANES, depth, f, (float)((v0.x >> L) << L) + hc,
                     (float)((v0.y >> L) << L) + hc, (float)((v0.z >> L) << L) + hc, tmin, tmax);
        if (BIG) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    tmin[k] = fminf(tmin[k], __shfl_xor(tmin[k], o, 64));
                    tmax[k] = fmaxf(tmax[k], __shfl_xor(tmax[k], o, 64));
                }
        }
        if (sub == 0) {
            uint64_t ob = w1 & 0x3FFFull;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float a0 = tmin[k] - slack, a1 = tmax[k] + slack;
                const int q0 = max((int)floorf(a0 / u), -128), q1 = min((int)ceilf(a1 / u), 127);
                ob |= (uint64_t)(uint8_t)(int8_t)q0 << (14 + 16 * k);
                ob |= (uint64_t)(uint8_t)(int8_t)q1 << (22 + 16 * k);
            }
            node[2 * t + 1] = ob;
        }
    }
}

// ----------------------------------------------------------------- search
// Visiting order of the 8 children: by the number of axes on which the child
// lies across from the query (0, 1, 1, 1, 2, 2, 2, 3).  Self-inverse.
__device__ __forceinline__ uint32_t near_order(uint32_t s) { return s == 3 ? 4u : (s == 4 ? 3u : s); }

// The child mask reordered by visiting slot: bit s of the result is bit
// near_order(s) ^ qo of m (XOR by qo swaps bit pairs, pair pairs, nibbles;
// near_order swaps slots 3 and 4).
__device__ __forceinline__ uint32_t slot_mask(uint32_t m, uint32_t qo) {
    if (qo & 1u) m = ((m & 0x55u) << 1) | ((m & 0xAAu) >> 1);
    if (qo & 2u) m = ((m & 0x33u) << 2) | ((m & 0xCCu) >> 2);
    if (qo & 4u) m = ((m & 0x0Fu) << 4) | ((m & 0xF0u) >> 4);
    return (m & 0xE7u) | ((m >> 1) & 0x08u) | ((m << 1) & 0x10u);
}

__device__ __forceinline__ uint32_t axis_gap(uint32_t q, uint32_t lo, uint32_t hi) {
    return q < lo ? lo - q : (q > hi ? q - hi : 0u);
}

__device__ __forceinline__ uint32_t isqrt64(uint64_t v) {
    uint64_t r = (uint64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (uint32_t)r;
}

// Team lane shifts for the shared candidate lists: a 64-bit value from the
// lane one below (DPP row shift; a team's lane 0 gets another team's value,
// which the caller discards), and one lane's value sent to every lane.
__device__ __forceinline__ uint32_t dpp_prev_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
}
__device__ __forceinline__ uint64_t dpp_prev_u64(uint64_t x) {
    return ((uint64_t)dpp_prev_u32((uint32_t)(x >> 32)) << 32) | dpp_prev_u32((uint32_t)x);
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Candidate lists of one query, shared by its team of knn_team<KT>() lanes: ascending
// in (squared distance, key index) over the team, lane t holding positions
// t*E .. t*E + E - 1 in registers (every array below is indexed only inside
// unrolled loops).  A candidate offered by one lane is sent to the whole team
// and inserted with one shift by one position: the team then prunes with the
// k-th distance of every candidate it has found.  Insertions need every lane
// of the team active.
//
// Up to depth 15 a squared voxel distance is below 2^32 - 1, so a candidate
// packs into one word, distance above index, whose integer order is the
// candidate order; distances are 32-bit throughout.
template <int KT>
struct PackedList {
    using Dist = uint32_t;
    static constexpr int kTeam = knn_team<KT>();
    static constexpr int E = KT >= kTeam ? KT / kTeam : 1;  // entries per lane
    static constexpr uint64_t kNone = ~0ull;  // bound meaning "no k-th candidate yet"
    struct Cand {
        uint64_t v;
    };
    uint64_t e[E];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int s = 0; s < E; ++s) e[s] = ~0ull;
    }
    __device__ static __forceinline__ Cand make(uint32_t d, int32_t i) {
        return Cand{((uint64_t)d << 32) | (uint32_t)i};
    }
    __device__ static __forceinline__ Cand bcast(Cand c, int src) { return Cand{shfl_u64(c.v, src)}; }
    // insert c (the same on every lane of the team); tl = lane within the team
    __device__ __forceinline__ void insert(Cand c, int tl) {
        const uint64_t v = c.v;
        const uint64_t p = dpp_prev_u64(e[E - 1]);
        const uint64_t below = tl == 0 ? 0ull : p;  // position t*E - 1 (none for lane 0)
#pragma unroll
        for (int s = E - 1; s > 0; --s) {
            const uint64_t lo = e[s - 1], cur = e[s];
            e[s] = v < lo ? lo : (v < cur ? v : cur);
        }
        e[0] = v < below ? below : (v < e[0] ? v : e[0]);
    }
    // the team's k-th distance, or kNone while it holds fewer than k; base =
    // the team's lane 0
    __device__ __forceinline__ uint64_t kth(int k, int base) const {
        const int pos = k - 1, slot = pos % E;
        uint32_t hi = (uint32_t)(e[0] >> 32);
#pragma unroll
        for (int s = 1; s < E; ++s) hi = s == slot ? (uint32_t)(e[s] >> 32) : hi;
        hi = (uint32_t)__shfl((int)hi, base + pos / E, 64);
        return hi == 0xFFFFFFFFu ? kNone : hi;
    }
    // this lane's entry s (team position tl*E + s)
    __device__ __forceinline__ void out(int s, int64_t &idx, uint64_t &d2) const {
        uint64_t v = e[0];
#pragma unroll
        for (int t = 1; t < E; ++t) v = t == s ? e[t] : v;
        idx = v == ~0ull ? -1 : (int64_t)(uint32_t)v;
        d2 = v == ~0ull ? ~0ull : (v >> 32);
    }
};

// Deeper grids: 64-bit distances beside the indexes, in two arrays (whole
// struct swaps would be lowered to memory copies).
template <int KT>
struct WideList {
    using Dist = uint64_t;
    static constexpr int kTeam = knn_team<KT>();
    static constexpr int E = KT >= kTeam ? KT / kTeam : 1;
    static constexpr uint64_t kNone = ~0ull;
    struct Cand {
        uint64_t d;
        int32_t i;
    };
    uint64_t d[E];
    int32_t i[E];
    __device__ static __forceinline__ bool less(uint64_t ad, int32_t ai, uint64_t bd, int32_t bi) {
        return ad < bd || (ad == bd && ai < bi);
    }
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            d[s] = ~0ull;
            i[s] = 0x7FFFFFFF;
        }
    }
    __device__ static __forceinline__ Cand make(uint64_t vd, int32_t vi) { return Cand{vd, vi}; }
    __device__ static __forceinline__ Cand bcast(Cand c, int src) {
        return Cand{shfl_u64(c.d, src), __shfl(c.i, src, 64)};
    }
    __device__ __forceinline__ void insert(Cand c, int tl) {
        const uint64_t vd = c.d;
        const int32_t vi = c.i;
        uint64_t bd = dpp_prev_u64(d[E - 1]);
        int32_t bi = (int32_t)dpp_prev_u32((uint32_t)i[E - 1]);
        if (tl == 0) {  // nothing below lane 0's first position
            bd = 0;
            bi = INT32_MIN;
        }
#pragma unroll
        for (int s = E - 1; s > 0; --s) {
            const bool sh = less(vd, vi, d[s - 1], i[s - 1]);
            const bool here = less(vd, vi, d[s], i[s]);
            const uint64_t nd = sh ? d[s - 1] : (here ? vd : d[s]);
            const int32_t ni = sh ? i[s - 1] : (here ? vi : i[s]);
            d[s] = nd;
            i[s] = ni;
        }
        const bool sh = less(vd, vi, bd, bi);
        const bool here = less(vd, vi, d[0], i[0]);
        const uint64_t nd = sh ? bd : (here ? vd : d[0]);
        const int32_t ni = sh ? bi : (here ? vi : i[0]);
        d[0] = nd;
        i[0] = ni;
    }
    __device__ __forceinline__ uint64_t kth(int k, int base) const {
        const int pos = k - 1, slot = pos % E;
        uint64_t m = d[0];
#pragma unroll
        for (int s = 1; s < E; ++s) m = s == slot ? d[s] : m;
        return shfl_u64(m, base + pos / E);
    }
    __device__ __forceinline__ void out(int s, int64_t &idx, uint64_t &d2) const {
        uint64_t vd = d[0];
        int32_t vi = i[0];
#pragma unroll
        for (int t = 1; t < E; ++t) {
            vd = t == s ? d[t] : vd;
            vi = t == s ? i[t] : vi;
        }
        idx = vd == ~0ull ? -1 : (int64_t)vi;
        d2 = vd;
    }
};

// Waves per SIMD the search is compiled for: five for packed lists up to
// k = 8 (94 VGPRs, no spills); 1 leaves the choice to the compiler (95 to
// 107 VGPRs, four or five waves, none spilling).
template <int KT, class LIST>
constexpr int knn_waves_per_eu() {
    return (KT <= 8 && sizeof(typename LIST::Dist) == 4) ? 5 : 1;
}

// One query at a time per team of knn_team<KT>() lanes: each team's first
// query by its place in the grid, the next ones from a counter (qctr, zero at
// launch; without it, round-robin over the grid).  LIST is PackedList (depth
// <= 15) or WideList.  The kernel is one loop whose every trip moves each
// team one step in its own query: set up a query, set up a round (its start
// cells), walk (one step per lane, with work handed from busy lanes to idle
// ones), end a round, so that a team whose query or round is over goes on
// with the next one instead of waiting for the other teams of its wave.
// kCount (a measurement build, same results): every lane counts its
// node-word loads, dense-table loads, voxels whose distance it took and walk
// steps, summed into work[0..3].
template <int KT, class LIST, bool kCount = false>
__global__ __launch_bounds__(kKnnBlock) __attribute__((amdgpu_waves_per_eu(knn_waves_per_eu<KT, LIST>())))
void k_knn_tree(
    const uint64_t *__restrict__ node, const uint32_t *__restrict__ dense,
    const int64_t *__restrict__ lvl, int64_t nodes_max, const float *__restrict__ q, int64_t nq,
    const uint64_t *__restrict__ order, float o0, float o1, float o2, float scale, uint32_t depth,
    int dl, int k, int la, int64_t *__restrict__ idx_out, uint64_t *__restrict__ d2_out,
    uint32_t *err, uint32_t *qctr, const uint32_t *__restrict__ perm = nullptr,
    unsigned long long *work = nullptr) {
    uint32_t c_node = 0, c_dense = 0, c_vox = 0, c_step = 0;  // kCount only
    using Dist = typename LIST::Dist;
    using Cand = typename LIST::Cand;
    // open node word per level 1 .. depth - 1 (the levels a walk opens),
    // one column per thread
    extern __shared__ uint64_t s_word[];
    __shared__ uint64_t s_sw[kKnnBlock], s_sc[kKnnBlock];  // start cells of the round: word, corner
    __shared__ int64_t s_base[kMaxDepth + 1];
    constexpr int kTeam = knn_team<KT>(), kTeamsPerBlock = kKnnBlock / kTeam;
    // (the list's lane shift is a DPP row shift: a team lies within a row of
    // 16 lanes)
    static_assert(kTeam >= kCells && kTeam <= 16 && (kTeam & (kTeam - 1)) == 0, "team size");
    const int tid = threadIdx.x, team = tid / kTeam, tl = tid % kTeam;
    const int tw = (tid & 63) / kTeam, tbase = (tid & 63) - tl;  // team within the wave, its lane 0
    const uint32_t tmask = (uint32_t)((1ull << kTeam) - 1ull);
    if (tid >= 1 && tid <= depth) s_base[tid] = lvl[kLvlBase + tid];
    __syncthreads();  // the only block-wide barrier; teams run independently after it
    // an oversized tree (keys that are not a CGA of the grid) searches nothing
    const int64_t n = tree_total(lvl) < 0 ? 0 : lvl[0];
    const int dt = dense_level(depth, dl);
    const float o[3] = {o0, o1, o2};
    const uint32_t top = (1u << depth) - 1;
    const int64_t stride = (int64_t)gridDim.x * kTeamsPerBlock;

    // ---- per query
    int64_t slot = (int64_t)blockIdx.x * kTeamsPerBlock + team, j = 0;
    uint32_t nxt = 0;  // lane 0: the team's next query from the counter, taken one query ahead
    auto next_slot = [&]() __attribute__((always_inline)) -> int64_t {
        return qctr ? stride + (int64_t)(uint32_t)__shfl((int)nxt, tbase, 64) : slot + stride;
    };
    Vox qv{0, 0, 0};
    uint64_t qkey = 0;
    LIST list;
    list.clear();
    uint64_t kth = LIST::kNone;  // the team's k-th distance
    bool round0 = true;
    uint32_t r = 0;
    int ls = 0;
    // Region already searched (a box of level-sk_l cells, every earlier
    // round's region inside it), skipped by later rounds so that the team's
    // list, kept from round to round, never takes a voxel twice.
    bool skip = false;
    int sk_l = 0;
    uint32_t sk_x0 = 0, sk_x1 = 0, sk_y0 = 0, sk_y1 = 0, sk_z0 = 0, sk_z1 = 0;
    // ---- per round: level of the walked subtrees, the start cells that
    // have this lane's child, that child's octant
    int l0 = 0;
    uint32_t avail = 0, qs = 0;
    // ---- per walk: depth-first, nearest child first.  The open node: its
    // level, corner and words (mask and first child; oriented box); the
    // query's octant one level down; the squared gap to the low and the high
    // child half on each axis (a child's box distance is then three selects
    // and two adds); whether its children are cells of the skipped level; the
    // bound, refreshed from the team's at every node, in the distance type
    // and saturated (every distance of a packed-list grid is below 2^32 - 1,
    // so "<=" keeps its meaning); its children within the bound at entry; the
    // slots still to visit.
    int l = -1;
    uint32_t x0 = 0, y0 = 0, z0 = 0;
    uint64_t w = 0, wo = 0;
    uint32_t qol = 0;
    Dist gxl = 0, gxh = 0, gyl = 0, gyh = 0, gzl = 0, gzh = 0;
    bool touch = false;
    Dist bnd = 0;
    uint32_t near = 0, pm = 0;
    // Work sharing within the team: lroot is the level this lane's walk
    // climbs back to (l0, or the node it took over); bit L of open marks an
    // ancestor at level L on its path that has children left after the one
    // walked, bit L of given one whose remaining children another lane took
    // over.
    int lroot = -1;
    uint32_t open = 0, given = 0;
    enum { kQuery, kRound, kWalk, kDone };
    int phase = kQuery;

    // the query's octant at level l is digit l of its Morton key
    auto qo = [&](int lv) __attribute__((always_inline)) -> uint32_t {
        return (uint32_t)(qkey >> (3 * lv)) & 7u;
    };
    auto box_dist = [&](uint32_t x, uint32_t y, uint32_t z, int lv) __attribute__((always_inline)) -> Dist {
        const uint32_t e = (1u << lv) - 1;
        const Dist gx = axis_gap(qv.x, x, x + e), gy = axis_gap(qv.y, y, y + e),
                   gz = axis_gap(qv.z, z, z + e);
        return gx * gx + gy * gy + gz * gz;
    };
    // a voxel's position: in the key array, or through perm in the caller's
    // LINEAR array (then ties go to the smaller LINEAR position, as there)
    auto cand = [&](Dist d, int32_t i) __attribute__((always_inline)) -> Cand {
        if (kCount) ++c_vox;
        return LIST::make(d, perm ? (int32_t)perm[i] : i);
    };
    auto skipped = [&](uint32_t x, uint32_t y, uint32_t z, int lv) __attribute__((always_inline)) {
        if (!skip || lv > sk_l) return false;
        x >>= sk_l;
        y >>= sk_l;
        z >>= sk_l;
        return x >= sk_x0 && x <= sk_x1 && y >= sk_y0 && y <= sk_y1 && z >= sk_z0 && z <= sk_z1;
    };
    // Node (index within its level) of the level-lv cell with corner (x, y,
    // z), or -1 if empty; at lv = 0 the key index of the voxel.
    auto find_node = [&](uint32_t x, uint32_t y, uint32_t z, int lv) __attribute__((always_inline)) -> int64_t {
        int L;
        int64_t nj;
        if (dt > 0 && lv <= dt) {
            const uint32_t v = dense[enc3(x >> dt, y >> dt, z >> dt, (uint32_t)dl, false)];
            if (kCount) ++c_dense;
            if (!v) return -1;
            nj = (int64_t)v - 1;
            L = dt;
        } else {
            nj = 0;  // the root
            L = (int)depth;
        }
        while (L > lv) {
            const uint64_t nw = node[2 * (s_base[L] + nj)];
            if (kCount) ++c_node;
            --L;
            const uint32_t oc = (((x >> L) & 1u) << 2) | (((y >> L) & 1u) << 1) | ((z >> L) & 1u);
            if (!((nw >> oc) & 1u)) return -1;
            nj = node_first(nw) + __popc((uint32_t)nw & 0xFFu & ((1u << oc) - 1u));
        }
        return nj;
    };
    auto to_dist = [](uint64_t b) __attribute__((always_inline)) -> Dist {
        return b > (uint64_t)(Dist)~(Dist)0 ? (Dist)~(Dist)0 : (Dist)b;
    };
    // Entering the open node (level l, corner x0, words w, wo): its child
    // gaps, the bound and the children within it.
    auto enter = [&](bool fresh) __attribute__((always_inline)) {
        const int cl = l - 1;
        qol = qo(cl);
        // gaps to the low half [0, h) and the high half [h, 2h) of the node
        // along an axis, each cut to the node's voxel box [blo, bhi], from
        // the query's signed offset t (every coordinate is below 2^21):
        // max(a - t, t - b, 0) over the cut interval [a, b] (an empty cut has
        // no child to visit)
        const int32_t h = 1 << cl;
        auto gaps = [&](int a, uint32_t qc, uint32_t c0, Dist &lo2, Dist &hi2) __attribute__((always_inline)) {
            uint32_t blo, bhi;
            node_box(w, a, l, blo, bhi);
            const int32_t t = (int32_t)(qc - c0);
            const int32_t la_ = (int32_t)blo, lb = min((int32_t)bhi, h - 1);
            const int32_t ha = max((int32_t)blo, h), hb = min((int32_t)bhi, 2 * h - 1);
            const int32_t gl = max(max(la_ - t, t - lb), 0), gh = max(max(ha - t, t - hb), 0);
            lo2 = (Dist)gl * (Dist)gl;
            hi2 = (Dist)gh * (Dist)gh;
        };
        gaps(0, qv.x, x0, gxl, gxh);
        gaps(1, qv.y, y0, gyl, gyh);
        gaps(2, qv.z, z0, gzl, gzh);
        touch = skip && cl == sk_l;
        bnd = to_dist(kth);
        // children already beyond the bound never take a step
        const Dist xl = gxl, xh = gxh;
        const Dist q0 = xl + gyl, q1 = xl + gyh, q2 = xh + gyl, q3 = xh + gyh;
        near = (q0 + gzl <= bnd ? 0x01u : 0u) | (q0 + gzh <= bnd ? 0x02u : 0u) |
               (q1 + gzl <= bnd ? 0x04u : 0u) | (q1 + gzh <= bnd ? 0x08u : 0u) |
               (q2 + gzl <= bnd ? 0x10u : 0u) | (q2 + gzh <= bnd ? 0x20u : 0u) |
               (q3 + gzl <= bnd ? 0x40u : 0u) | (q3 + gzh <= bnd ? 0x80u : 0u);
        // a node just loaded whose oriented box lies beyond the bound opens
        // no child (rounded up, the bound only keeps more); tested in rounds
        // from cells of level kObbMinLevel up, those of queries far from the
        // voxels (near ones, settled in smaller rounds, would pay for the
        // test and rarely gain: on the 2 x 10M sphere points, rounds from
        // smaller cells pruned one node load per thousand with it)
        if (fresh && near && !round0 && ls >= kObbMinLevel) {
            const float hc = (float)((1u << l) - 1u) * 0.5f;
            const float lb2 = obb_dist2(wo, l, (float)qv.x - ((float)x0 + hc),
                                        (float)qv.y - ((float)y0 + hc), (float)qv.z - ((float)z0 + hc));
            if (lb2 > (float)bnd * (1.f + 1.f / 1048576.f) + 1.f) near = 0;
        }
    };

    uint32_t trip = 0;
    for (;;) {
        ++trip;
        bool pend = false;  // this lane's voxel for the team's list, if any
        Cand cv{};
        // ---- next query of the team
        if (phase == kQuery) {
            if (slot >= nq) {
                phase = kDone;
            } else {
                if (qctr && tl == 0) nxt = atomicAdd(qctr, 1u);
                j = order ? (int64_t)(order[slot] >> kOrderBits) : slot;  // query (and output row)
                const bool finite = quantize3(q[3 * j], q[3 * j + 1], q[3 * j + 2], o, scale, depth, qv);
                if (!finite && tl == 0) set_err(err, ERR_NONFINITE);
                if (!finite || n == 0) {
                    for (int s = tl; s < k; s += kTeam) {
                        idx_out[j * k + s] = -1;
                        d2_out[j * k + s] = ~0ull;
                    }
                    slot = next_slot();
                } else {
                    qkey = enc3(qv.x, qv.y, qv.z, depth, false);
                    list.clear();
                    kth = LIST::kNone;
                    skip = false;
                    round0 = true;
                    r = 0;
                    ls = la - 1;
                    phase = kRound;
                }
            }
        }
        // ---- next round: this lane's start cell (round 0: one child of the
        // query's level-la cell; later rounds: one of the level-ls cells
        // covering the cube [q - r, q + r], the query's own cell and, per
        // axis where the cube crosses a cell border, the neighbour)
        if (phase == kRound) {
            uint32_t c[3];
            bool ok = tl < kCells;  // the team's lanes beyond the eight cells start idle
            {
                const uint32_t c3[3] = {qv.x, qv.y, qv.z};
                if (round0) {
                    const uint32_t oc = near_order((uint32_t)tl & 7u) ^ qo(la - 1);
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        c[a] = ((c3[a] >> la) << la) | (((oc >> (2 - a)) & 1u) << (la - 1));
                } else {
                    const uint32_t m = near_order((uint32_t)tl & 7u);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const uint32_t lo = c3[a] > r ? c3[a] - r : 0;
                        const uint32_t hi = (uint64_t)c3[a] + r < top ? c3[a] + r : top;
                        const uint32_t own = c3[a] >> ls, clo = lo >> ls, chi = hi >> ls;
                        if ((m >> (2 - a)) & 1u) {
                            const uint32_t other = own == clo ? chi : clo;
                            ok = ok && other != own;
                            c[a] = other << ls;
                        } else {
                            c[a] = own << ls;
                        }
                    }
                }
            }
            const int64_t cn = ok && !skipped(c[0], c[1], c[2], ls) ? find_node(c[0], c[1], c[2], ls) : -1;
            // The start cells are shared out a child at a time: lane tl walks
            // child near_order(tl) ^ (query octant) of every start cell in
            // turn, so that the heaviest cell's work is spread over the team.
            // Start cells at level 0 are voxels: each is offered by its lane.
            l0 = ls - 1;
            avail = 0;
            if (ls == 0) {
                if (cn >= 0) {
                    const Dist d = box_dist(c[0], c[1], c[2], 0);
                    if (d <= kth) {
                        pend = true;
                        cv = cand(d, (int32_t)cn);
                    }
                }
            } else {
                s_sw[tid] = cn >= 0 ? node[2 * (s_base[ls] + cn)] : 0ull;
                if (kCount) c_node += cn >= 0 ? 1u : 0u;
                s_sc[tid] = (uint64_t)c[0] | ((uint64_t)c[1] << 21) | ((uint64_t)c[2] << 42);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                qs = near_order((uint32_t)tl & 7u) ^ qo(l0);
#pragma unroll
                for (int m = 0; m < kCells; ++m) avail |= (uint32_t)((s_sw[team * kTeam + m] >> qs) & 1u) << m;
                if (tl >= kCells) avail = 0;
            }
            l = l0;
            lroot = l0;
            pm = 0;
            open = 0;
            given = 0;
            phase = kWalk;
        }
        // ---- one walk step: take over work, start this lane's next subtree,
        // climb back to the parent (its slots up to the one just finished are
        // done), or take the next child -- prune it, offer it (a voxel), or
        // descend into it.  Taking over, starting, climbing and descending
        // share one node-entry tail, so a wave whose lanes take different
        // paths runs it once.
        if (phase == kWalk) {
            // A lane without work left takes the remaining children of the
            // shallowest open ancestor of a lane that has one (the k-th idle
            // lane of the team pairs with its k-th such lane), every other
            // trip (each hand-over costs the wave about 40 instructions; on
            // every trip the 1M-query search took 3 % longer).  A team's
            // lanes move in step, so no atomics are needed.
            bool recv = false;
            int rsrc = 0, rl = 0;
            uint32_t rx = 0, ry = 0, rz = 0;
            {
                const bool idle = pm == 0 && l == lroot && !avail;
                const uint32_t ti = (uint32_t)(__ballot(idle) >> (kTeam * tw)) & tmask;
                const uint32_t td = (uint32_t)(__ballot(open != 0) >> (kTeam * tw)) & tmask;
                if ((trip & 1u) && __ballot(ti != 0 && td != 0)) {
                    const uint32_t below = (1u << tl) - 1u;
                    const int np = min(__popc(ti), __popc(td));
                    const int gl = open ? 31 - __builtin_clz(open) : 0;
                    if (open && __popc(td & below) < np) {
                        given |= 1u << gl;
                        open &= ~(1u << gl);
                    }
                    const int ri = __popc(ti & below);
                    uint32_t m = td;
#pragma unroll
                    for (int i = 0; i < kTeam - 1; ++i)
                        if (i < ri) m &= m - 1u;
                    rsrc = m ? __builtin_ctz(m) : tl;
                    rl = __shfl(gl, tbase + rsrc, 64);
                    rx = (uint32_t)__shfl((int)x0, tbase + rsrc, 64);
                    ry = (uint32_t)__shfl((int)y0, tbase + rsrc, 64);
                    rz = (uint32_t)__shfl((int)z0, tbase + rsrc, 64);
                    recv = idle && ri < np;
                }
            }
            const bool up = pm == 0;
            bool moved = false, climbed = false;
            uint32_t done_oc = 0;
            if (recv) {
                // enter the ancestor as if climbing back into it from the
                // child the other lane is walking
                l = rl;
                lroot = rl;
                done_oc = (((rx >> (l - 1)) & 1u) << 2) | (((ry >> (l - 1)) & 1u) << 1) | ((rz >> (l - 1)) & 1u);
                const uint32_t clr = ~((1u << l) - 1u);
                x0 = rx & clr;
                y0 = ry & clr;
                z0 = rz & clr;
                w = s_word[(l - 1) * kKnnBlock + (tid - tl + rsrc)];
                s_word[(l - 1) * kKnnBlock + tid] = w;
                moved = climbed = true;
            } else if (up && l == lroot && !avail) {
                // nothing left: wait for a hand-over or the end of the round
            } else if (up && l == lroot) {
                if (kCount) ++c_step;
                const int m = __builtin_ctz(avail);
                avail &= avail - 1;
                const uint64_t sw = s_sw[team * kTeam + m], sc = s_sc[team * kTeam + m];
                const uint32_t cx = ((uint32_t)sc & 0x1FFFFFu) | (((qs >> 2) & 1u) << l0);
                const uint32_t cy = ((uint32_t)(sc >> 21) & 0x1FFFFFu) | (((qs >> 1) & 1u) << l0);
                const uint32_t cz = ((uint32_t)(sc >> 42) & 0x1FFFFFu) | ((qs & 1u) << l0);
                const int32_t ci = (int32_t)node_first(sw) + __popc((uint32_t)sw & 0xFFu & ((1u << qs) - 1u));
                const Dist bd = box_dist(cx, cy, cz, l0);
                if (bd <= kth && !skipped(cx, cy, cz, l0)) {
                    if (l0 == 0) {
                        pend = true;
                        cv = cand(bd, ci);
                    } else {
                        const u64x2 pr = *(const u64x2 *)(node + 2 * (s_base[l0] + ci));
                        w = pr.x;
                        wo = pr.y;
                        if (kCount) ++c_node;
                        s_word[(l0 - 1) * kKnnBlock + tid] = w;
                        x0 = cx;
                        y0 = cy;
                        z0 = cz;
                        moved = true;
                    }
                }
            } else if (up) {
                if (kCount) ++c_step;
                done_oc = (((x0 >> l) & 1u) << 2) | (((y0 >> l) & 1u) << 1) | ((z0 >> l) & 1u);
                ++l;
                open &= ~(1u << l);
                const uint32_t clr = ~((1u << l) - 1u);
                x0 &= clr;
                y0 &= clr;
                z0 &= clr;
                w = s_word[(l - 1) * kKnnBlock + tid];
                moved = climbed = true;
            } else {
                if (kCount) ++c_step;
                const uint32_t sl = __builtin_ctz(pm);
                pm &= pm - 1;
                const uint32_t oc = near_order(sl) ^ qol;
                const Dist bd = ((oc & 4u) ? gxh : gxl) + ((oc & 2u) ? gyh : gyl) + ((oc & 1u) ? gzh : gzl);
                const int cl = l - 1;
                const uint32_t cx = x0 | (((oc >> 2) & 1u) << cl), cy = y0 | (((oc >> 1) & 1u) << cl),
                               cz = z0 | ((oc & 1u) << cl);
                if (bd <= bnd && !(touch && skipped(cx, cy, cz, cl))) {
                    const int32_t ci = (int32_t)node_first(w) + __popc((uint32_t)w & 0xFFu & ((1u << oc) - 1u));
                    if (cl == 0) {
                        pend = true;
                        cv = cand(bd, ci);
                    } else {
                        const u64x2 pr = *(const u64x2 *)(node + 2 * (s_base[cl] + ci));
                        w = pr.x;
                        wo = pr.y;
                        if (kCount) ++c_node;
                        s_word[(cl - 1) * kKnnBlock + tid] = w;
                        if (pm) open |= 1u << l;
                        l = cl;
                        x0 = cx;
                        y0 = cy;
                        z0 = cz;
                        moved = true;
                    }
                }
            }
            if (moved) {
                enter(!climbed);
                const uint32_t done_slots = climbed ? (2u << near_order(done_oc ^ qol)) - 1u : 0u;
                pm = slot_mask((uint32_t)w & near, qol) & ~done_slots;
                if (climbed && ((given >> l) & 1u)) {  // its remaining children went to another lane
                    pm = 0;
                    given &= ~(1u << l);
                }
            }
        }
        // ---- the team's list takes what its lanes offered, one lane after
        // another; the team's k-th distance follows (every lane of a team is
        // active here)
        {
            const uint64_t b = __ballot(pend);
            if (b) {
                uint32_t tm = (uint32_t)(b >> (kTeam * tw)) & tmask;
                while (tm) {
                    const int src = __builtin_ctz(tm);
                    tm &= tm - 1;
                    list.insert(LIST::bcast(cv, tbase + src), tl);
                }
                kth = list.kth(k, tbase);
                bnd = kth < (uint64_t)bnd ? to_dist(kth) : bnd;
            }
        }
        // ---- end of a round: every lane of a walking team is out of work
        const bool busy = phase == kWalk && !(pm == 0 && l == lroot && !avail);
        if (phase == kWalk && !((uint32_t)(__ballot(busy) >> (kTeam * tw)) & tmask)) {
            // Exact once every voxel within the k-th distance lies in the
            // region searched so far: the pruning only ever used k-th
            // distances of real candidates, so no voxel of that ball inside
            // the region was missed.
            bool done;
            if (round0) {
                // every voxel outside the level-la cell is at least m away
                const uint32_t c3[3] = {qv.x, qv.y, qv.z};
                uint64_t m = ~0ull;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const uint32_t b = (c3[a] >> la) << la;
                    const uint64_t below = (uint64_t)(c3[a] - b) + 1, above = (uint64_t)b + (1u << la) - c3[a];
                    if (b > 0 && below < m) m = below;
                    if ((uint64_t)b + (1u << la) <= top && above < m) m = above;
                }
                done = m == ~0ull || (kth != LIST::kNone && m * m > kth);
            } else {
                done = (kth != LIST::kNone && isqrt64(kth) <= r) || ls == (int)depth;
            }
            if (done) {
#pragma unroll
                for (int s = 0; s < LIST::E; ++s) {
                    const int pos = tl * LIST::E + s;
                    if (pos < k) {
                        int64_t idx;
                        uint64_t d2;
                        list.out(s, idx, d2);
                        idx_out[j * k + pos] = idx;
                        d2_out[j * k + pos] = d2;
                    }
                }
                slot = next_slot();
                phase = kQuery;
            } else {
                // the region just searched is skipped from now on
                skip = true;
                if (round0) {
                    sk_l = la;
                    sk_x0 = sk_x1 = qv.x >> la;
                    sk_y0 = sk_y1 = qv.y >> la;
                    sk_z0 = sk_z1 = qv.z >> la;
                } else {
                    sk_l = ls;
                    sk_x0 = (qv.x > r ? qv.x - r : 0) >> ls;
                    sk_y0 = (qv.y > r ? qv.y - r : 0) >> ls;
                    sk_z0 = (qv.z > r ? qv.z - r : 0) >> ls;
                    sk_x1 = ((uint64_t)qv.x + r < top ? qv.x + r : top) >> ls;
                    sk_y1 = ((uint64_t)qv.y + r < top ? qv.y + r : top) >> ls;
                    sk_z1 = ((uint64_t)qv.z + r < top ? qv.z + r : top) >> ls;
                }
                const uint64_t bound = kth;
                // next cube: the k-th distance ball, or a grown cube while
                // fewer than k candidates are known (from round 0 at least one
                // level-la cell wide, so that the next region contains the la
                // cell)
                if (bound != LIST::kNone) r = isqrt64(bound);
                else if (round0) r = ((1u << la) - 1) / 2 > 1 ? ((1u << la) - 1) / 2 : 1;
                else r = 2 * r + 1;
                if (r > top) r = top;
                ls = 0;
                while (ls < (int)depth && (1u << ls) < 2 * r + 1) ++ls;
                round0 = false;
                phase = kRound;
            }
        }
        if (!__ballot(phase != kDone)) break;
    }
    if (kCount) {  // the team's sums, one atomic per counter per team
#pragma unroll
        for (int o2 = 1; o2 < kTeam; o2 <<= 1) {
            c_node += __shfl_xor(c_node, o2, 64);
            c_dense += __shfl_xor(c_dense, o2, 64);
            c_vox += __shfl_xor(c_vox, o2, 64);
            c_step += __shfl_xor(c_step, o2, 64);
        }
        if (tl == 0 && (c_node | c_dense | c_vox | c_step)) {
            atomicAdd(&work[0], (unsigned long long)c_node);
            atomicAdd(&work[1], (unsigned long long)c_dense);
            atomicAdd(&work[2], (unsigned long long)c_vox);
            atomicAdd(&work[3], (unsigned long long)c_step);
        }
    }
}

// LINEAR keys -> the Morton keys of the same voxels, with each key's position.
template <typename K>
__global__ __launch_bounds__(256) void k_linear_to_morton(const K *__restrict__ keys, int64_t n_host,
                                                          const int64_t *d_n, uint32_t depth,
                                                          K *__restrict__ mk, uint32_t *__restrict__ pos) {
    const int64_t n = key_count(n_host, d_n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Vox v = dec3((uint64_t)keys[i], depth, true);
        mk[i] = (K)enc3(v.x, v.y, v.z, depth, false);
        pos[i] = (uint32_t)i;
    }
}

// Ordering code of every query: its index above the top kOrderBits of its
// Morton key, with the digit histogram of the three 8-bit passes.
__global__ __launch_bounds__(256) void k_knn_order(const float *__restrict__ q, int64_t nq, float o0,
                                                   float o1, float o2, float scale,
                                                   uint32_t depth, uint64_t *__restrict__ out,
                                                   uint32_t *hist) {
    constexpr int RB = 8, PASSES = kOrderBits / RB;
    __shared__ uint32_t s_h[PASSES << RB];
    for (int i = threadIdx.x; i < (PASSES << RB); i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const float o[3] = {o0, o1, o2};
    const int drop = 3 * (int)depth > kOrderBits ? 3 * (int)depth - kOrderBits : 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x) {
        Vox v;
        quantize3(q[3 * i], q[3 * i + 1], q[3 * i + 2], o, scale, depth, v);  // the search reports non-finite queries
        const uint64_t code = ((uint64_t)i << kOrderBits) | (enc3(v.x, v.y, v.z, depth, false) >> drop);
        out[i] = code;
        hist_add<RB>(s_h, code, PASSES);
    }
    __syncthreads();
    hist_flush<RB>(s_h, hist, PASSES);
}

// Launch knob (never changes results): CGA_KNN_LA = level of the round-0 cell.
static int knn_la(uint32_t depth) {
    int la = kLaDefault;
    if (const char *e = getenv("CGA_KNN_LA")) {
        const int v = atoi(e);
        if (v >= 1 && v <= kMaxDepth) la = v;
    }
    return la < (int)depth ? la : (int)depth;
}

// Launch knob (never changes results): CGA_KNN_ORDER = 1 / 0 forces the query
// ordering on / off; by default it is on from kOrderMin queries.
static bool knn_order(int64_t nq) {
    if (const char *e = getenv("CGA_KNN_ORDER")) return atoi(e) != 0 && nq > 0;
    return nq >= kOrderMin;
}

// Launch knob (never changes results): CGA_KNN_QUEUE = 1 / 0 forces the
// search's query counter on / off; by default it is on from
// kKnnQueuePerTeam queries per resident team.
static int knn_queue_knob() {
    if (const char *e = getenv("CGA_KNN_QUEUE")) return atoi(e) != 0 ? 1 : 0;
    return -1;
}

// Launch knob (never changes results): CGA_KNN_BLOCKS = n caps the search's
// grid at n blocks, so that every team answers many queries in turn.
static int knn_blocks_knob() {
    if (const char *e = getenv("CGA_KNN_BLOCKS")) return atoi(e);
    return 0;
}

// Upper bound on the number of octree nodes of n unique keys: level L has at
// most min(n, 8^(depth - L)) nodes.
static int64_t tree_nodes_max(int64_t n, uint32_t depth) {
    int64_t t = 0;
    for (uint32_t L = 1; L <= depth; ++L) {
        const uint32_t e = 3 * (depth - L);
        const int64_t cap = e >= 62 ? INT64_MAX : (int64_t)1 << e;
        t += n < cap ? n : cap;
    }
    return t > 0 ? t : 1;
}

struct KnnLayout {
    Control *ctl;
    SortWs sort;             // query ordering (when on)
    uint64_t *oa = nullptr, *ob = nullptr;
    uint32_t *cnt;
    int64_t *lvl;
    uint32_t *first;
    uint8_t *oct;
    uint64_t *node;
    float *mom;        // build-time moments of each node's voxels
    uint32_t *kfirst;  // each node's first key
    uint32_t *big;     // nodes of more than kSmallNode keys, one level at a time
    // LINEAR keys only: their Morton re-keys (in, alternate, sorted) with
    // the key positions riding along, and the sort's workspace
    SortWs msort;
    void *mk[3] = {nullptr, nullptr, nullptr};
    uint32_t *pos[3] = {nullptr, nullptr, nullptr};
    const uint32_t *perm = nullptr;  // set per call: the sorted keys' LINEAR positions
    uint32_t *dense;
    int dl;  // levels spanned by the dense table
    int64_t tiles, nodes;
    size_t bytes;
};

static KnnLayout knn_layout(void *ws, int64_t n, uint32_t depth, int64_t nq_order = 0,
                            bool linear = false) {
    KnnLayout L;
    Carve c(ws);
    L.tiles = n > 0 ? (n + kTreeTile - 1) / kTreeTile : 1;
    L.nodes = tree_nodes_max(n, depth);
    L.ctl = c.take<Control>(1);
    if (linear) {  // LINEAR keys: re-keyed to Morton and sorted with their positions
        SortCfg cfg;
        cfg.radix_bits = 8;
        cfg.items = 16;
        sort_carve(c, L.msort, n, 3 * (int)depth, cfg);
        const size_t kb = wide_keys(depth) ? 8 : 4, m = (size_t)(n > 0 ? n : 1);
        for (int b = 0; b < 3; ++b) L.mk[b] = c.take<uint8_t>(m * kb);
        for (int b = 0; b < 3; ++b) L.pos[b] = c.take<uint32_t>(m);
    }
    if (nq_order > 0) {
        SortCfg cfg;
        cfg.radix_bits = 8;
        cfg.items = 16;
        sort_carve(c, L.sort, nq_order, kOrderBits, cfg);
        L.oa = c.take<uint64_t>((size_t)nq_order);
        L.ob = c.take<uint64_t>((size_t)nq_order);
    }
    L.lvl = c.take<int64_t>(kLvlWords);
    L.cnt = c.take<uint32_t>((size_t)L.tiles * depth);
    L.first = c.take<uint32_t>((size_t)L.nodes);
    L.oct = c.take<uint8_t>((size_t)L.nodes);
    L.node = c.take<uint64_t>(2 * (size_t)L.nodes);  // two words per node
    L.mom = c.take<float>(10 * (size_t)L.nodes);
    L.kfirst = c.take<uint32_t>((size_t)L.nodes);
    L.big = c.take<uint32_t>((size_t)(n / kSmallNode + 1));
    L.dl = dense_levels(n);
    L.dense = c.take<uint32_t>((size_t)dense_cells(depth, L.dl) + 1);
    L.bytes = c.size();
    return L;
}

template <typename K>
static void tree_build(const KnnLayout &L, const K *keys, int64_t n, const int64_t *d_n,
                       uint32_t depth, hipStream_t s, const char *label = "knn_tree",
                       bool emit = false, uint8_t *occ = nullptr, int64_t occ_cap = 0,
                       int64_t *counts = nullptr) {
    CGA_PROF(label, s);
    const int dt = dense_level(depth, L.dl);
    k_tree_count<K><<<(unsigned)L.tiles, 256, 0, s>>>(keys, n, d_n, depth, L.tiles, L.cnt, L.dense,
                                                      dense_cells(depth, L.dl), &L.ctl->err);
    k_tree_scan<<<depth, 1024, 0, s>>>(L.cnt, L.tiles, n, d_n, L.lvl);
    k_tree_bases<<<1, 64, 0, s>>>(L.lvl, depth, L.nodes);
    k_tree_build<K><<<(unsigned)L.tiles, 256, 0, s>>>(keys, n, d_n, depth, dt, L.tiles, L.cnt, L.lvl,
                                                      L.first, L.kfirst, L.oct, L.dense,
                                                      dense_cells(depth, L.dl), L.nodes);
    for (uint32_t lev = 1; lev <= depth; ++lev) {
        // level lev holds at most min(n, 8^(depth - lev)) nodes
        const uint32_t e = 3 * (depth - lev);
        const int64_t cap = e >= 62 ? INT64_MAX : (int64_t)1 << e;
        // latency-bound passes (a thread per node walks its children):
        // many blocks in flight; their set-up is two parallel loads
        int64_t blocks = ((n < cap ? n : cap) + 255) / 256;
        blocks = blocks < 1 ? 1 : (blocks < 4096 ? blocks : 4096);
        k_tree_mask<K><<<(unsigned)blocks, 256, 0, s>>>(keys, depth, lev, L.lvl, L.first, L.oct,
                                                        L.node, L.mom, L.nodes, emit, occ, occ_cap,
                                                        counts, &L.ctl->err);
        if (lev >= 2 && (int)lev <= kScanLevels) {
            const int64_t m = n < cap ? n : cap;
            int64_t tb = (m + 255) / 256, wb = (m / kSmallNode + 3) / 4;  // at most m / 16 big nodes
            tb = tb < 1 ? 1 : (tb < 4096 ? tb : 4096);
            wb = wb < 1 ? 1 : (wb < 2048 ? wb : 2048);
            uint32_t *n_big = &L.ctl->tile_ctr[kTreeBigCtr + lev];
            k_tree_ranges<K, false><<<(unsigned)tb, 256, 0, s>>>(keys, depth, lev, L.lvl, L.kfirst,
                                                                 L.node, L.big, n_big);
            k_tree_ranges<K, true><<<(unsigned)wb, 256, 0, s>>>(keys, depth, lev, L.lvl, L.kfirst,
                                                                L.node, L.big, n_big);
        }
    }
}

// Blocks of the search kernel resident on the whole GPU at once (occupancy
// per CU times the CU count; no cap if the runtime cannot say), cached per
// kernel, LDS size and device.
template <int KT>
static int64_t knn_resident_blocks(bool packed, bool counting, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<bool, bool, size_t, int>, int64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return INT64_MAX;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(packed, counting, lds, dev);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    hipError_t e;
    if (packed)
        e = counting ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_knn_tree<KT, PackedList<KT>, true>, kKnnBlock, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_knn_tree<KT, PackedList<KT>, false>, kKnnBlock, lds);
    else
        e = counting ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_knn_tree<KT, WideList<KT>, true>, kKnnBlock, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_knn_tree<KT, WideList<KT>, false>, kKnnBlock, lds);
    if (e != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        per_cu = cus = 0;
    const int64_t b = (int64_t)per_cu * cus;
    cache[key] = b > 0 ? b : INT64_MAX;
    return cache[key];
}

template <int KT, bool kCount = false>
static void knn_launch(const cga_grid *g, const KnnLayout &L, const float *q, int64_t nq, int k,
                       int64_t *idx, uint64_t *d2, hipStream_t s,
                       unsigned long long *work = nullptr) {
    CGA_PROF(kCount ? "knn_count" : "knn", s);
    const size_t lds = (size_t)(g->depth > 1 ? g->depth - 1 : 1) * kKnnBlock * sizeof(uint64_t);
    // as many blocks as the GPU holds at once (each team then goes on from
    // query to query), fewer for small query sets
    constexpr int kTeamsPerBlock = kKnnBlock / knn_team<KT>();
    const int64_t want = (nq + kTeamsPerBlock - 1) / kTeamsPerBlock;
    int64_t cap = knn_resident_blocks<KT>(g->depth <= kPackedDepth, kCount, lds);
    if (const int b = knn_blocks_knob(); b > 0 && b < cap) cap = b;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
    // Teams take their queries from a counter (zeroed with the control block
    // at the call's start) when each has many to take: a slow query then
    // holds up only its own team.  With few queries per team the counter's
    // atomics would contend (100k queries over 2 x 1M LiDAR points: 1.21
    // against 0.80 ms), and each team takes every grid-stride'th query.  The
    // counter's 32 bits must not wrap.
    const int64_t teams = (int64_t)blocks * kTeamsPerBlock;
    const int knob = knn_queue_knob();
    const bool queue = knob >= 0 ? knob == 1 : nq >= kKnnQueuePerTeam * teams;
    uint32_t *qctr = queue && nq < (int64_t)UINT32_MAX - teams ? &L.ctl->tile_ctr[kKnnQueryCtr] : nullptr;
    if (g->depth <= kPackedDepth)
        k_knn_tree<KT, PackedList<KT>, kCount><<<blocks, kKnnBlock, lds, s>>>(
            L.node, L.dense, L.lvl, L.nodes, q, nq, L.ob, g->origin[0], g->origin[1], g->origin[2],
            g->scale, g->depth, L.dl, k, knn_la(g->depth), idx, d2, &L.ctl->err, qctr, L.perm, work);
    else
        k_knn_tree<KT, WideList<KT>, kCount><<<blocks, kKnnBlock, lds, s>>>(
            L.node, L.dense, L.lvl, L.nodes, q, nq, L.ob, g->origin[0], g->origin[1], g->origin[2],
            g->scale, g->depth, L.dl, k, knn_la(g->depth), idx, d2, &L.ctl->err, qctr, L.perm, work);
}

template <bool kCount>
static void knn_dispatch(const cga_grid *g, const KnnLayout &L, const float *q, int64_t nq, int k,
                         int64_t *idx, uint64_t *d2, hipStream_t s, unsigned long long *work) {
    if (k <= 1) knn_launch<1, kCount>(g, L, q, nq, k, idx, d2, s, work);
    else if (k <= 2) knn_launch<2, kCount>(g, L, q, nq, k, idx, d2, s, work);
    else if (k <= 4) knn_launch<4, kCount>(g, L, q, nq, k, idx, d2, s, work);
    else if (k <= 8) knn_launch<8, kCount>(g, L, q, nq, k, idx, d2, s, work);
    else if (k <= 16) knn_launch<16, kCount>(g, L, q, nq, k, idx, d2, s, work);
    else knn_launch<32, kCount>(g, L, q, nq, k, idx, d2, s, work);
}

// ---------------------------------------------------------- binary lookup
__global__ __launch_bounds__(256) void k_binary_lookup(const uint64_t *__restrict__ keys,
                                                       int64_t n_host, const int64_t *d_n,
                                                       const uint64_t *__restrict__ q, int64_t nq,
                                                       int64_t *__restrict__ rank,
                                                       uint8_t *__restrict__ found) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nq) return;
    const int64_t n = dev_count(n_host, d_n);
    const uint64_t v = q[j];
    const int64_t r = lower_bound_dev(keys, n, v);
    rank[j] = r;
    if (found) found[j] = (uint8_t)(r < n && keys[r] == v);
}

// LINEAR keys: their Morton re-keys sorted with the key positions (an 8-bit
// key-value radix sort: mk[0] -> ... -> mk[2], pos likewise); the tree is
// built over mk[2] and the search reports positions through pos[2].
template <typename K>
static void linear_rekey(KnnLayout &L, const K *keys, int64_t n, const int64_t *d_n,
                         uint32_t depth, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    {
        CGA_PROF("knn_rekey", s);
        k_linear_to_morton<K><<<(unsigned)blocks, 256, 0, s>>>(keys, n, d_n, depth, (K *)L.mk[0],
                                                                L.pos[0]);
    }
    sort_launch_kv<K>(L.msort, (const K *)L.mk[0], (K *)L.mk[2], (K *)L.mk[1], (K *)L.mk[2],
                      L.pos[0], L.pos[2], L.pos[1], L.pos[2], n, d_n, false,
                      &L.ctl->tile_ctr[kLinearSortCtr], s);
    L.perm = L.pos[2];
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_knn_workspace_bytes(const cga_grid *g, int64_t n, int64_t nq) {
    if (!grid_valid(g) || n < 0 || nq < 0) return 0;
    return knn_layout(nullptr, n, g->depth, knn_order(nq) ? nq : 0,
                      g->key_mode == CGA_KEY_LINEAR).bytes;
}


static int knn_call(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                    const float *d_q, int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2, void *d_ws,
                    size_t ws_bytes, cga_stream stream, unsigned long long *work) {
    if (!grid_valid(g) || n < 0 || n > INT32_MAX || nq < 0 || k < 1 || k > 32 || !d_ws)
        return CGA_EINVAL;
    if (nq > 0 && (!d_q || !d_idx || !d_d2)) return CGA_EINVAL;
    if (n > 0 && !d_keys) return CGA_EINVAL;
    if (nq >= ((int64_t)1 << (64 - kOrderBits))) return CGA_EUNSUPPORTED;
    const bool ordered = knn_order(nq), linear = g->key_mode == CGA_KEY_LINEAR;
    KnnLayout L = knn_layout(d_ws, n, g->depth, ordered ? nq : 0, linear);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(L.ctl, ordered ? L.sort.hist : nullptr, ordered ? sort_zero_bytes(L.sort) : 0,
                         linear ? L.msort.hist : nullptr, linear ? sort_zero_bytes(L.msort) : 0,
                         nullptr, s));
    if (nq > 0) {
        if (ordered) {
            int64_t blocks = (nq + 256 * 8 - 1) / (256 * 8);
            blocks = blocks > 1024 ? 1024 : blocks;
            {
                CGA_PROF("knn_order", s);
                k_knn_order<<<(unsigned)blocks, 256, 0, s>>>(d_q, nq, g->origin[0], g->origin[1],
                                                              g->origin[2], g->scale, g->depth, L.oa,
                                                              L.sort.hist);
            }
            // three passes: oa -> ob -> oa -> ob
            sort_launch<uint64_t>(L.sort, L.oa, L.ob, L.oa, L.ob, nq, nullptr, true,
                                  L.ctl->tile_ctr, s);
        } else {
            L.ob = nullptr;
        }
        const void *tk = d_keys;  // the keys the tree is built over (Morton order)
        if (linear && n > 0) {
            if (wide_keys(g->depth))
                linear_rekey<uint64_t>(L, (const uint64_t *)d_keys, n, d_n, g->depth, s);
            else
                linear_rekey<uint32_t>(L, (const uint32_t *)d_keys, n, d_n, g->depth, s);
            tk = L.mk[2];
        }
        if (wide_keys(g->depth))
            tree_build<uint64_t>(L, (const uint64_t *)tk, n, d_n, g->depth, s);
        else
            tree_build<uint32_t>(L, (const uint32_t *)tk, n, d_n, g->depth, s);
        if (work) knn_dispatch<true>(g, L, d_q, nq, k, d_idx, d_d2, s, work);
        else knn_dispatch<false>(g, L, d_q, nq, k, d_idx, d_d2, s, nullptr);
        CGA_HIP(hipGetLastError());
    }
    return CGA_OK;
}

int cga_knn(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n, const float *d_q,
            int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2, void *d_ws, size_t ws_bytes,
            cga_stream stream) {
    return knn_call(g, d_keys, n, d_n, d_q, nq, k, d_idx, d_d2, d_ws, ws_bytes, stream, nullptr);
}

int cga_knn_count(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                  const float *d_q, int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2,
                  uint64_t *d_work, void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!d_work) return CGA_EINVAL;
    return knn_call(g, d_keys, n, d_n, d_q, nq, k, d_idx, d_d2, d_ws, ws_bytes, stream,
                    (unsigned long long *)d_work);
}

size_t cga_occupancy_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    return knn_layout(nullptr, n, g->depth).bytes;
}

int cga_occupancy(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint8_t *d_occ, int64_t occ_cap, int64_t *d_counts, void *d_ws, size_t ws_bytes,
                  cga_stream stream) {
    if (!grid_valid(g) || n < 0 || n > INT32_MAX || occ_cap < 0 || !d_ws) return CGA_EINVAL;
    if ((n > 0 && !d_keys) || (occ_cap > 0 && !d_occ)) return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_MORTON) return CGA_EUNSUPPORTED;
    KnnLayout L = knn_layout(d_ws, n, g->depth);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(L.ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (wide_keys(g->depth))
        tree_build<uint64_t>(L, (const uint64_t *)d_keys, n, d_n, g->depth, s, "occupancy", true,
                             d_occ, occ_cap, d_counts);
    else
        tree_build<uint32_t>(L, (const uint32_t *)d_keys, n, d_n, g->depth, s, "occupancy", true,
                             d_occ, occ_cap, d_counts);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

int cga_binary_lookup(const uint64_t *d_keys, int64_t n, const int64_t *d_n, const uint64_t *d_q,
                      int64_t nq, int64_t *d_rank, uint8_t *d_found, cga_stream stream) {
    if (n < 0 || nq < 0) return CGA_EINVAL;
    if ((n > 0 && !d_keys) || (nq > 0 && (!d_q || !d_rank))) return CGA_EINVAL;
    if (nq == 0) return CGA_OK;
    hipStream_t s = (hipStream_t)stream;
    CGA_PROF("binary_lookup", s);
    k_binary_lookup<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(d_keys, n, d_n, d_q, nq, d_rank,
                                                                d_found);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
