// Batched CGA construction of F frames and the union of every consecutive
// frame pair, sized entirely on the device so the whole sequence can be
// captured once in a hipGraph and replayed:
//   1. quantize + encode every point as the composite key (frame << 3d | key)
//      with the digit histograms of the sort on the side;
//   2. an LSD radix sort segmented by frame: each frame's keys sorted on
//      their own, in place of the frame's range, by the 3 * depth key bits
//      only (with very many frames, one sort of the composite keys);
//   3. run-length compaction -> unique composite keys + point counts;
//   4. per-frame offsets (binary search of each frame's first key) and the
//      frame bits stripped off;
//   5. pair set-up: each pair's merged capacity, output start and its number
//      of merge windows, as prefix sums;
//   6. one persistent merge kernel whose workgroups pull windows of all
//      F - 1 pairs from one queue (merge path + dedupe + look-back inside
//      each pair).
// Plus the sort autotuner, which times every compiled digit width and tile
// size on real or synthetic keys and remembers the fastest.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "cga_common.h"
#include "cga_merge.h"
#include "cga_rle.h"
#include "cga_sort.h"

namespace cga {

SortCfg default_sort_cfg(bool wide, int64_t n, int key_bits);

// ------------------------------------------------------------ tuning cache
namespace {
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::map<std::tuple<int, int, int>, SortCfg> g_tune;  // (key bytes, key bits, log2 n) -> cfg

int log2_bucket(int64_t n) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << (b + 1)) <= n) ++b;
    return b;
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("CGA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    int kb, bits, lg, rb, items;
    while (fscanf(f, "%d %d %d %d %d", &kb, &bits, &lg, &rb, &items) == 5) {
        SortCfg c;
        c.radix_bits = rb;
        c.items = items;
        if (sort_cfg_supported(c)) g_tune[std::make_tuple(kb, bits, lg)] = c;  // malformed lines ignored
    }
    fclose(f);
}

void tune_store_locked(int kb, int bits, int lg, const SortCfg &c) {
    g_tune[std::make_tuple(kb, bits, lg)] = c;
    const char *path = getenv("CGA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %d %d %d\n", kb, bits, lg, c.radix_bits, c.items);
    fclose(f);
}
}  // namespace

// The configuration for a sort: the caller's, else a tuned one, else default.
bool tuned_sort_cfg(int key_bytes, int key_bits, int64_t n, SortCfg *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(std::make_tuple(key_bytes, key_bits, log2_bucket(n)));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

static int resolve_cfg(const cga_tune *t, int key_bytes, int key_bits, int64_t n, SortCfg *out) {
    if (t) {
        SortCfg c;
        c.radix_bits = (int)t->radix_bits;
        c.items = (int)t->tile_items;
        if (!sort_cfg_supported(c)) return CGA_EINVAL;
        *out = c;
        return CGA_OK;
    }
    if (!tuned_sort_cfg(key_bytes, key_bits, n, out)) *out = default_sort_cfg(key_bytes == 8, n, key_bits);
    return CGA_OK;
}

// ----------------------------------------------------------------- kernels
// Frame of point i: the last f with off[f] <= i (off has F + 1 entries).
__device__ __forceinline__ uint32_t frame_of(const int64_t *off, int F, int64_t i) {
    int lo = 0, len = F;
    while (len > 1) {
        const int half = len >> 1;
        lo = off[lo + half] <= i ? lo + half : lo;
        len -= half;
    }
    return (uint32_t)lo;
}

// Block b encodes the points [b * chunk, (b + 1) * chunk), frame by frame,
// and adds the digits of every sort pass to LDS counters that it flushes at
// each frame's end: into hist[p][f][digit] for a segmented sort (seg), else
// into the one histogram hist[p][digit] of the composite keys.
template <int RB>
__global__ __launch_bounds__(256) void k_batch_encode(const float *__restrict__ xyz,
                                                      const int64_t *__restrict__ off, int F,
                                                      int64_t n, int64_t chunk, float o0, float o1,
                                                      float o2, float scale, uint32_t depth,
                                                      int linear, uint64_t *__restrict__ keys,
                                                      int passes, int seg, uint32_t *hist,
                                                      uint32_t *err) {
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_h[];
    __shared__ int s_bad;
    const uint32_t nh = (uint32_t)passes * RADIX;
    for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) s_h[i] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const float o[3] = {o0, o1, o2};
    const int shift = 3 * (int)depth;
    bool bad = false;
    int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    uint32_t f = c0 < c1 ? frame_of(off, F, c0) : (uint32_t)F;
    while (c0 < c1) {
        const int64_t fe = off[f + 1], e = fe < c1 ? fe : c1;
        for (int64_t i = c0 + threadIdx.x; i < e; i += blockDim.x) {
            Vox v;
            bad |= !quantize3(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], o, scale, depth, v);
            const uint64_t k = ((uint64_t)f << shift) | enc3(v.x, v.y, v.z, depth, linear != 0);
            keys[i] = k;
            hist_add_coherent<RB>(s_h, k, passes);
        }
        __syncthreads();
        if (e > c0) {
            for (uint32_t j = threadIdx.x; j < nh; j += blockDim.x) {
                const uint32_t c = s_h[j];
                if (c) {
                    const uint32_t p = j / RADIX, d = j % RADIX;
                    atomicAdd(&hist[seg ? ((size_t)p * F + f) * RADIX + d : j], c);
                    s_h[j] = 0;
                }
            }
        }
        __syncthreads();
        c0 = e;
        ++f;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_bad) set_err(err, ERR_NONFINITE);
}

template <typename K>
__device__ __forceinline__ int64_t lower_bound_u(const K *keys, int64_t n, uint64_t q) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((uint64_t)keys[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// key_off[f] = first unique composite key of frame >= f, f = 0..F.
__global__ void k_batch_offsets(const uint64_t *__restrict__ comp, const int64_t *d_u, int F,
                                int shift, int64_t *__restrict__ key_off) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > F) return;
    key_off[f] = lower_bound_u(comp, *d_u, (uint64_t)f << shift);
}

template <typename K>
__global__ void k_batch_strip(const uint64_t *__restrict__ comp, const int64_t *d_u, uint64_t mask,
                              K *__restrict__ out) {
    const int64_t u = *d_u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < u;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (K)(comp[i] & mask);
}

// Pair p = (frame p, frame p + 1): merged capacity, output start, windows.
// One block; a serial prefix over chunks of blockDim pairs.
__global__ void k_batch_pairs(const int64_t *__restrict__ key_off, int F,
                              int64_t *__restrict__ merged_off, int64_t *__restrict__ tile_off,
                              int64_t *total_tiles) {
    __shared__ int64_t s_w[1024 / 64];
    __shared__ int64_t s_base;
    const int P = F - 1;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < P; c0 += blockDim.x) {
        const int p = c0 + threadIdx.x;
        int64_t tiles = 0;
        if (p < P) {
            const int64_t tot = key_off[p + 2] - key_off[p];  // U_p + U_{p+1}
            tiles = (tot + kMergeTile - 1) / kMergeTile;
            merged_off[p] = key_off[p] + key_off[p + 1] - key_off[1];
        }
        int64_t tot_tiles;
        const int64_t ex = block_excl_sum<1024>(tiles, s_w, &tot_tiles);
        if (p < P) tile_off[p] = s_base + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_base += tot_tiles;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total_tiles = s_base;
        if (P >= 0) tile_off[P > 0 ? P : 0] = s_base;  // sentinel after the last pair
    }
}

// Pair of merge window `tile`: the last p with tile_off[p] <= tile.
__device__ __forceinline__ int pair_of(const int64_t *tile_off, int P, int64_t tile) {
    int lo = 0, len = P;
    while (len > 1) {
        const int half = len >> 1;
        lo = tile_off[lo + half] <= tile ? lo + half : lo;
        len -= half;
    }
    return lo;
}

// part[tile] = A elements before the window's first diagonal, one thread
// per window, all windows at once (the merge loop below would otherwise
// wait for two dependent searches per window).
template <typename K>
__global__ void k_batch_partition(const K *__restrict__ keys, const int64_t *__restrict__ key_off,
                                  int F, const int64_t *__restrict__ tile_off,
                                  const int64_t *total_tiles, int64_t *__restrict__ part) {
    const int64_t T = *total_tiles;
    for (int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tile < T;
         tile += (int64_t)gridDim.x * blockDim.x) {
        const int p = pair_of(tile_off, F - 1, tile);
        const int64_t na = key_off[p + 1] - key_off[p], nb = key_off[p + 2] - key_off[p + 1];
        part[tile] = merge_path(keys + key_off[p], na, keys + key_off[p + 1], nb,
                                (tile - tile_off[p]) * kMergeTile);
    }
}

// Persistent: workgroups take windows from one queue until all pairs are done.
template <typename K>
__global__ __launch_bounds__(kMergeBlock) void k_batch_merge(
    const K *__restrict__ keys, const int64_t *__restrict__ key_off, int F,
    const int64_t *__restrict__ merged_off, const int64_t *__restrict__ tile_off,
    const int64_t *total_tiles, const int64_t *__restrict__ part, K *__restrict__ merged,
    int64_t *__restrict__ merged_cnt, uint64_t *status, uint32_t *tile_ctr, uint32_t *err) {
    __shared__ uint32_t s_tile;
    __shared__ MergeShared<K> sh;
    const int64_t T = *total_tiles;
    const int P = F - 1;
    for (;;) {
        const int64_t tile = (int64_t)next_tile(tile_ctr, &s_tile);
        if (tile >= T) break;  // uniform across the workgroup
        const int p = pair_of(tile_off, P, tile);
        const int64_t first_tile = tile_off[p];
        const K *A = keys + key_off[p];
        const K *B = keys + key_off[p + 1];
        const int64_t na = key_off[p + 1] - key_off[p], nb = key_off[p + 2] - key_off[p + 1];
        const int64_t d0 = (tile - first_tile) * kMergeTile;
        const int64_t d1 = d0 + kMergeTile < na + nb ? d0 + kMergeTile : na + nb;
        // a window that does not end its pair is followed by the pair's next
        const int64_t a0 = part[tile], a1 = d1 == na + nb ? na : part[tile + 1];
        __syncthreads();  // the previous window's use of sh is over
        const int64_t cap = na + nb;
        merge_tile<K>(sh, A, na, B, nb, d0, d1, a0, a1, merged + merged_off[p], nullptr, cap,
                      merged_cnt + p, status, tile, first_tile, err);
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------ layout
struct BatchLayout {
    Control *ctl;
    SortWs sort;
    uint64_t *rle_status;
    uint64_t *buf_a, *buf_b;
    int64_t *tile_off, *total_tiles;
    uint64_t *merge_status;
    int64_t *merge_part;
    int64_t merge_tiles_bound;
    int frame_bits;
    bool seg;  // each frame sorted on its own by its 3 * depth key bits
    size_t bytes;
};

static int frame_bits_of(int F) {
    int b = 0;
    while ((1 << b) < F) ++b;
    return b;
}

// Up to this many frames the sort is segmented by frame: the frames are
// already in order, so only the 3 * depth key bits take passes, not the
// frame bits above them.  Beyond it (many small frames: many part-filled
// tiles, large per-frame histograms) one sort of the composite keys.
constexpr int kSegMaxFrames = 4096;

static bool batch_segmented(int F) { return F <= kSegMaxFrames; }

// Key bits the sort passes cover (and the autotuner is asked about).
static int batch_sort_bits(const cga_grid *g, int F) {
    return 3 * (int)g->depth + (batch_segmented(F) ? 0 : frame_bits_of(F));
}

static BatchLayout batch_layout(void *ws, const cga_grid *g, int F, int64_t n, const SortCfg &cfg) {
    BatchLayout L;
    Carve c(ws);
    L.frame_bits = frame_bits_of(F);
    L.seg = batch_segmented(F);
    L.ctl = c.take<Control>(1);
    sort_carve(c, L.sort, n, batch_sort_bits(g, F), cfg, L.seg ? F : 0);
    L.rle_status = c.take<uint64_t>((size_t)rle_tiles(n));
    L.buf_a = c.take<uint64_t>((size_t)(n > 0 ? n : 1));
    L.buf_b = c.take<uint64_t>((size_t)(n > 0 ? n : 1));
    L.tile_off = c.take<int64_t>((size_t)F + 1);
    L.total_tiles = c.take<int64_t>(1);
    L.merge_tiles_bound = (2 * n + kMergeTile - 1) / kMergeTile + F + 1;
    L.merge_status = c.take<uint64_t>((size_t)L.merge_tiles_bound);
    L.merge_part = c.take<int64_t>((size_t)L.merge_tiles_bound);
    L.bytes = c.size();
    return L;
}

static int persistent_groups() {
    static int groups = 0;
    if (!groups) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        groups = cus * 4;
    }
    return groups;
}

template <int RB>
static void batch_encode_launch(const cga_grid *g, const float *xyz, const int64_t *off, int F,
                                int64_t n, uint64_t *keys, int passes, bool seg, uint32_t *hist,
                                uint32_t *err, hipStream_t s) {
    int64_t blocks = (n + 256 * 8 - 1) / (256 * 8);
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    int64_t chunk = (n + blocks - 1) / blocks;
    chunk = (chunk + 255) / 256 * 256;
    CGA_PROF("batch_encode", s);
    k_batch_encode<RB><<<(unsigned)blocks, 256, hist_lds_bytes(passes, RB), s>>>(
        xyz, off, F, n, chunk, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth,
        g->key_mode == CGA_KEY_LINEAR, keys, passes, seg ? 1 : 0, hist, err);
}

static void batch_encode_dispatch(int rb, const cga_grid *g, const float *xyz, const int64_t *off,
                                  int F, int64_t n, uint64_t *keys, int passes, bool seg,
                                  uint32_t *hist, uint32_t *err, hipStream_t s) {
    switch (rb) {
        case 4: batch_encode_launch<4>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 5: batch_encode_launch<5>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 6: batch_encode_launch<6>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 7: batch_encode_launch<7>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 9: batch_encode_launch<9>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 10: batch_encode_launch<10>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        case 11: batch_encode_launch<11>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
        default: batch_encode_launch<8>(g, xyz, off, F, n, keys, passes, seg, hist, err, s); break;
    }
}

struct BatchArgs {
    cga_grid g;
    const float *xyz;
    const int64_t *off;
    int F;
    int64_t n;
    void *keys;
    uint32_t *counts;
    int64_t *key_off;
    void *merged;
    int64_t *merged_off, *merged_cnt;
    void *ws;
    size_t ws_bytes;
    SortCfg cfg;
};

static int batch_validate(const cga_grid *g, const float *xyz, const int64_t *off, int F,
                          int64_t n, void *keys, int64_t *key_off, void *merged,
                          int64_t *merged_off, int64_t *merged_cnt, void *ws) {
    if (!grid_valid(g) || F < 1 || F > 65536 || n < 0 || !off || !key_off || !ws)
        return CGA_EINVAL;
    if (n > 0 && (!xyz || !keys)) return CGA_EINVAL;
    if (F > 1 && (!merged || !merged_off || !merged_cnt)) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    if (3 * (int)g->depth + frame_bits_of(F) > 64) return CGA_EUNSUPPORTED;
    return CGA_OK;
}

template <typename K>
static int batch_enqueue(const BatchArgs &a, hipStream_t s) {
    BatchLayout L = batch_layout(a.ws, &a.g, a.F, a.n, a.cfg);
    if (a.ws_bytes < L.bytes) return CGA_EWORKSPACE;
    const int shift = 3 * (int)a.g.depth;
    CGA_TRY(launch_begin(L.ctl, L.sort.hist, sort_zero_bytes(L.sort), L.merge_status,
                         (size_t)L.merge_tiles_bound * 8, nullptr, s));
    {
        // the rle status and the tail of the pair arrays start at zero too
        int64_t nz = (int64_t)(rle_tiles(a.n));
        k_fill_i64<<<64, 256, 0, s>>>((int64_t *)L.rle_status, nz, 0);
    }
    const int64_t n = a.n;
    int64_t *d_u = &L.ctl->count;
    if (n > 0) {
        batch_encode_dispatch(L.sort.radix_bits, &a.g, a.xyz, a.off, a.F, n, L.buf_a, L.sort.passes,
                              L.seg, L.sort.hist, &L.ctl->err, s);
        uint64_t *fin = (L.sort.passes & 1) ? L.buf_b : L.buf_a;
        uint64_t *other = (L.sort.passes & 1) ? L.buf_a : L.buf_b;
        if (L.seg)
            sort_launch_seg(L.sort, L.buf_a, fin, other, fin, a.off, L.ctl->tile_ctr, s);
        else
            sort_launch<uint64_t>(L.sort, L.buf_a, fin, other, fin, n, nullptr, true,
                                  L.ctl->tile_ctr, s);
        // unique composite keys go to the buffer the sort did not end in
        {
            CGA_PROF("rle", s);
            k_rle<uint64_t, uint64_t, false><<<(unsigned)rle_tiles(n), kRleBlock, 0, s>>>(
                fin, n, nullptr, 0, ~0ull, other, a.counts, nullptr, n, d_u, L.rle_status,
                &L.ctl->tile_ctr[kMaxPasses], &L.ctl->err);
        }
        {
            CGA_PROF("batch_offsets", s);
            k_batch_offsets<<<(unsigned)((a.F + 1 + 255) / 256), 256, 0, s>>>(other, d_u, a.F, shift,
                                                                            a.key_off);
            const uint64_t mask = shift >= 64 ? ~0ull : ((1ull << shift) - 1);
            int64_t blocks = (n + 255) / 256;
            blocks = blocks > 2048 ? 2048 : blocks;
            k_batch_strip<K><<<(unsigned)blocks, 256, 0, s>>>(other, d_u, mask, (K *)a.keys);
        }
    } else {
        k_fill_i64<<<1, 256, 0, s>>>(a.key_off, a.F + 1, 0);
    }
    if (a.F > 1) {
        {
            CGA_PROF("batch_pairs", s);
            k_batch_pairs<<<1, 1024, 0, s>>>(a.key_off, a.F, a.merged_off, L.tile_off, L.total_tiles);
            k_fill_i64<<<1, 256, 0, s>>>(a.merged_cnt, a.F - 1, 0);
        }
        int64_t groups = persistent_groups();
        groups = groups < L.merge_tiles_bound ? groups : L.merge_tiles_bound;
        int64_t pblocks = (L.merge_tiles_bound + 255) / 256;
        pblocks = pblocks > 4096 ? 4096 : pblocks;
        CGA_PROF("batch_merge", s);
        k_batch_partition<K><<<(unsigned)pblocks, 256, 0, s>>>((const K *)a.keys, a.key_off, a.F,
                                                              L.tile_off, L.total_tiles, L.merge_part);
        k_batch_merge<K><<<(unsigned)groups, kMergeBlock, 0, s>>>(
            (const K *)a.keys, a.key_off, a.F, a.merged_off, L.tile_off, L.total_tiles,
            L.merge_part, (K *)a.merged, a.merged_cnt, L.merge_status,
            &L.ctl->tile_ctr[kMaxPasses + 1], &L.ctl->err);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

static int batch_run(const BatchArgs &a, hipStream_t s) {
    return wide_keys(a.g.depth) ? batch_enqueue<uint64_t>(a, s) : batch_enqueue<uint32_t>(a, s);
}

struct BatchGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

// --------------------------------------------------------------- autotuner
template <typename K>
__global__ void k_tune_copy(const K *in, int64_t n, K *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

template <typename K>
__global__ void k_tune_keys(K *keys, int64_t n, uint32_t bits, uint64_t seed) {
    const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;  // splitmix64 finaliser
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        keys[i] = (K)((z ^ (z >> 31)) & mask);
    }
}

// Time one candidate: fill `src` (the caller's keys or synthetic ones), then
// the best of three full sorts.
template <typename K>
static int tune_one(const SortWs &w, Control *ctl, const K *user, int64_t n, uint32_t bits, K *src,
                    K *a, K *b, hipEvent_t e0, hipEvent_t e1, hipStream_t s, float *tmin) {
    if (user) k_tune_copy<K><<<1024, 256, 0, s>>>(user, n, src);
    else k_tune_keys<K><<<1024, 256, 0, s>>>(src, n, bits, 12345);
    *tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        CGA_TRY(launch_begin(ctl, w.hist, sort_zero_bytes(w), nullptr, 0, nullptr, s));
        CGA_HIP(hipEventRecord(e0, s));
        sort_launch<K>(w, src, b, a, b, n, nullptr, false, ctl->tile_ctr, s);
        CGA_HIP(hipEventRecord(e1, s));
        CGA_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CGA_HIP(hipEventElapsedTime(&ms, e0, e1));
        *tmin = ms < *tmin ? ms : *tmin;
    }
    return CGA_OK;
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_batch_workspace_bytes(const cga_grid *g, int nframes, int64_t n) {
    if (!grid_valid(g) || nframes < 1 || n < 0) return 0;
    size_t m = 0;
    for (int rb = 4; rb <= 11; ++rb)
        for (int items : kSortItems) {
            SortCfg c;
            c.radix_bits = rb;
            c.items = items;
            size_t b = batch_layout(nullptr, g, nframes, n, c).bytes;
            m = b > m ? b : m;
        }
    return m;
}

int cga_batch_sort_bits(const cga_grid *g, int nframes) {
    if (!grid_valid(g) || nframes < 1 || nframes > 65536) return 0;
    return batch_sort_bits(g, nframes);
}

int cga_batch_build_merge(const cga_grid *g, const float *d_xyz, const int64_t *d_off, int nframes,
                          int64_t n, void *d_keys, uint32_t *d_counts, int64_t *d_key_off,
                          void *d_merged, int64_t *d_merged_off, int64_t *d_merged_cnt,
                          const cga_tune *tune, void *d_ws, size_t ws_bytes, cga_stream stream) {
    CGA_TRY(batch_validate(g, d_xyz, d_off, nframes, n, d_keys, d_key_off, d_merged, d_merged_off,
                           d_merged_cnt, d_ws));
    BatchArgs a{*g, d_xyz, d_off, nframes, n, d_keys, d_counts, d_key_off, d_merged, d_merged_off,
                d_merged_cnt, d_ws, ws_bytes, SortCfg()};
    CGA_TRY(resolve_cfg(tune, 8, batch_sort_bits(g, nframes), n, &a.cfg));
    return batch_run(a, (hipStream_t)stream);
}

int cga_batch_graph_create(const cga_grid *g, const float *d_xyz, const int64_t *d_off,
                           int nframes, int64_t n, void *d_keys, uint32_t *d_counts,
                           int64_t *d_key_off, void *d_merged, int64_t *d_merged_off,
                           int64_t *d_merged_cnt, const cga_tune *tune, void *d_ws,
                           size_t ws_bytes, void **graph_out) {
    if (!graph_out) return CGA_EINVAL;
    *graph_out = nullptr;
    CGA_TRY(batch_validate(g, d_xyz, d_off, nframes, n, d_keys, d_key_off, d_merged, d_merged_off,
                           d_merged_cnt, d_ws));
    BatchArgs a{*g, d_xyz, d_off, nframes, n, d_keys, d_counts, d_key_off, d_merged, d_merged_off,
                d_merged_cnt, d_ws, ws_bytes, SortCfg()};
    CGA_TRY(resolve_cfg(tune, 8, batch_sort_bits(g, nframes), n, &a.cfg));
    if (ws_bytes < batch_layout(nullptr, g, nframes, n, a.cfg).bytes) return CGA_EWORKSPACE;
    persistent_groups();  // query the device before capture
    hipStream_t cs;
    CGA_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    BatchGraph *bg = new BatchGraph();
    int st = CGA_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = batch_run(a, cs);
        e = hipStreamEndCapture(cs, &bg->graph);
        if (e == hipSuccess && st == CGA_OK) e = hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0);
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || st != CGA_OK) {
        if (bg->exec) (void)hipGraphExecDestroy(bg->exec);
        if (bg->graph) (void)hipGraphDestroy(bg->graph);
        delete bg;
        if (e != hipSuccess) {
            g_last_hip_error = (int)e;
            return CGA_EHIP;
        }
        return st;
    }
    *graph_out = bg;
    return CGA_OK;
}

int cga_batch_graph_launch(void *graph, cga_stream stream) {
    if (!graph) return CGA_EINVAL;
    CGA_HIP(hipGraphLaunch(((BatchGraph *)graph)->exec, (hipStream_t)stream));
    return CGA_OK;
}

int cga_batch_graph_destroy(void *graph) {
    if (!graph) return CGA_OK;
    BatchGraph *bg = (BatchGraph *)graph;
    if (bg->exec) (void)hipGraphExecDestroy(bg->exec);
    if (bg->graph) (void)hipGraphDestroy(bg->graph);
    delete bg;
    return CGA_OK;
}

size_t cga_autotune_workspace_bytes(uint32_t key_bytes, int64_t n) {
    if ((key_bytes != 4 && key_bytes != 8) || n < 0) return 0;
    size_t m = 0;
    for (int rb = 4; rb <= 11; ++rb)
        for (int items : kSortItems) {
            SortCfg c;
            c.radix_bits = rb;
            c.items = items;
            Carve cv(nullptr);
            cv.take<Control>(1);
            SortWs w;
            sort_carve(cv, w, n, 64, c);
            for (int b = 0; b < 3; ++b) cv.take<uint64_t>((size_t)(n > 0 ? n : 1));
            m = cv.size() > m ? cv.size() : m;
        }
    return m;
}

int cga_autotune_sort(const void *d_keys, uint32_t key_bytes, uint32_t key_bits, int64_t n,
                      void *d_ws, size_t ws_bytes, cga_tune *best, float *best_ms,
                      cga_stream stream) {
    if ((key_bytes != 4 && key_bytes != 8) || key_bits < 1 || key_bits > 8 * key_bytes || n < 1 ||
        !d_ws)
        return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    if (ws_bytes < cga_autotune_workspace_bytes(key_bytes, n)) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    CGA_HIP(hipEventCreate(&e0));
    CGA_HIP(hipEventCreate(&e1));
    SortCfg best_cfg = default_sort_cfg(key_bytes == 8, n, (int)key_bits);
    float best_t = 1e30f;
    int status = CGA_OK;
    for (int rb = 4; rb <= 11 && status == CGA_OK; ++rb)
        for (int items : kSortItems) {
            SortCfg c;
            c.radix_bits = rb;
            c.items = items;
            Carve cv(d_ws);
            Control *ctl = cv.take<Control>(1);
            SortWs w;
            sort_carve(cv, w, n, (int)key_bits, c);
            void *src = cv.take<uint64_t>((size_t)n);
            void *a = cv.take<uint64_t>((size_t)n), *b = cv.take<uint64_t>((size_t)n);
            float tmin = 1e30f;
            status = key_bytes == 8
                         ? tune_one<uint64_t>(w, ctl, (const uint64_t *)d_keys, n, key_bits,
                                              (uint64_t *)src, (uint64_t *)a, (uint64_t *)b, e0, e1,
                                              s, &tmin)
                         : tune_one<uint32_t>(w, ctl, (const uint32_t *)d_keys, n, key_bits,
                                              (uint32_t *)src, (uint32_t *)a, (uint32_t *)b, e0, e1,
                                              s, &tmin);
            if (status != CGA_OK) break;
            if (tmin < best_t) {
                best_t = tmin;
                best_cfg = c;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != CGA_OK) return status;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        tune_store_locked((int)key_bytes, (int)key_bits, log2_bucket(n), best_cfg);
    }
    if (best) {
        best->radix_bits = (uint32_t)best_cfg.radix_bits;
        best->tile_items = (uint32_t)best_cfg.items;
    }
    if (best_ms) *best_ms = best_t;
    return CGA_OK;
}

}  // extern "C"
