// LSD radix sort of voxel keys for gfx950: one upfront histogram of every
// digit, then one "onesweep" kernel per digit (Adinets & Merrill, 2022): each
// workgroup ranks a tile of keys by digit with wave64 ballots, finds the
// global position of each of its digit buckets by a decoupled look-back over
// the tiles before it (Merrill & Garland, 2016), stages the tile in LDS in
// digit order and scatters it.  Stable, so passes compose.
#pragma once

#include <type_traits>

#include "cga_common.h"

namespace cga {

// No payload: the keys alone are sorted.  A payload type V (uint32_t) moves
// with its key through every pass (a key-value sort).
struct NoVal {};

constexpr int kSortBlock = 256;
constexpr int kMaxPasses = 16;  // 64 bits at 4 bits per digit

// Look-back status word: 2-bit flag + 30-bit count.
constexpr int kLookWindow = 8;  // predecessors read per look-back round trip
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;

struct SortCfg {
    int radix_bits = 8;
    int items = 16;
};

inline int sort_passes(int key_bits, int radix_bits) {
    return key_bits <= 0 ? 0 : (key_bits + radix_bits - 1) / radix_bits;
}
inline int64_t sort_tiles(int64_t n, int items) {
    int64_t t = (int64_t)kSortBlock * items;
    return n <= 0 ? 1 : (n + t - 1) / t;
}

// ------------------------------------------------------------ histogram
// Adds key's digits of every pass into LDS counters s_h[p][digit].
template <int RB, typename K>
__device__ __forceinline__ void hist_add(uint32_t *s_h, K key, int passes) {
    constexpr uint32_t RADIX = 1u << RB;
    for (int p = 0; p < passes; ++p) {
        uint32_t d = (uint32_t)(key >> (p * RB)) & (RADIX - 1);
        atomicAdd(&s_h[p * RADIX + d], 1u);
    }
}

// hist_add for keys of neighbouring points (an encode in input order, a
// re-key of sorted keys): where the active lanes of the wave share a digit,
// as the high digits of neighbouring keys mostly do, one add of their number
// replaces theirs.  On unordered keys the check only costs.
template <int RB, typename K>
__device__ __forceinline__ void hist_add_coherent(uint32_t *s_h, K key, int passes) {
    constexpr uint32_t RADIX = 1u << RB;
    const uint64_t act = __ballot(1);
    const int leader = __ffsll((unsigned long long)act) - 1;
    for (int p = 0; p < passes; ++p) {
        uint32_t d = (uint32_t)(key >> (p * RB)) & (RADIX - 1);
        const uint32_t d0 = __shfl(d, leader, 64);
        if (__ballot(d == d0) == act) {
            if (lane_id() == leader) atomicAdd(&s_h[p * RADIX + d0], (uint32_t)__popcll(act));
        } else {
            atomicAdd(&s_h[p * RADIX + d], 1u);
        }
    }
}

template <int RB>
__device__ __forceinline__ void hist_flush(const uint32_t *s_h, uint32_t *g_h, int passes) {
    constexpr uint32_t RADIX = 1u << RB;
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += blockDim.x) {
        uint32_t c = s_h[i];
        if (c) atomicAdd(&g_h[i], c);
    }
}

template <typename K, int RB>
__global__ __launch_bounds__(kSortBlock) void k_histogram(const K *__restrict__ in, int64_t n_host,
                                                          const int64_t *d_n, int passes,
                                                          uint32_t *__restrict__ hist) {
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_h[];
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const int64_t n = dev_count(n_host, d_n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        hist_add<RB>(s_h, in[i], passes);
    __syncthreads();
    hist_flush<RB>(s_h, hist, passes);
}

// Exclusive scan of each pass's histogram in place (one block per pass).
// Segmented (nseg > 0): hist[p][f][digit] per pass and segment, one block
// per (pass, segment), and each scan starts at the segment's first index
// seg_off[f], so it gives every digit's first output slot directly.
template <int RB>
__global__ __launch_bounds__(kSortBlock) void k_hist_scan(uint32_t *hist,
                                                          const int64_t *seg_off = nullptr,
                                                          int nseg = 0) {
    constexpr int RADIX = 1 << RB;
    constexpr int DPT = RADIX > kSortBlock ? RADIX / kSortBlock : 1;
    __shared__ uint32_t s_w[kSortBlock / 64];
    uint32_t *h = hist + (size_t)blockIdx.x * RADIX;
    const uint32_t start = nseg > 0 ? (uint32_t)seg_off[blockIdx.x % nseg] : 0u;
    uint32_t v[DPT], sum = 0;
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        int d = t * DPT + j;
        v[j] = d < RADIX ? h[d] : 0u;
        sum += v[j];
    }
    uint32_t tot;
    uint32_t ex = start + block_excl_sum<kSortBlock>(sum, s_w, &tot);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        int d = t * DPT + j;
        if (d < RADIX) h[d] = ex;
        ex += v[j];
    }
}

// Segments of consecutive keys, seg_off[0..nseg] (seg_off[nseg] = n), each
// cut into its own tiles of `tile` keys: seg_tiles[f] = first tile of
// segment f, seg_tiles[nseg] = the number of tiles.  One block of BLOCK.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_seg_tiles(const int64_t *__restrict__ seg_off, int nseg,
                                                     int64_t tile, int64_t *__restrict__ seg_tiles) {
    __shared__ int64_t s_w[BLOCK / 64];
    int64_t carry = 0;
    for (int f0 = 0; f0 < nseg; f0 += BLOCK) {
        const int f = f0 + (int)threadIdx.x;
        const int64_t len = f < nseg ? seg_off[f + 1] - seg_off[f] : 0;
        const int64_t t = (len + tile - 1) / tile;
        int64_t tot;
        const int64_t ex = block_excl_sum<BLOCK>(t, s_w, &tot);
        if (f < nseg) seg_tiles[f] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) seg_tiles[nseg] = carry;
}

// --------------------------------------------------------- onesweep pass
// One LSD pass on digit bits [shift, shift + RB).  `look` holds one status
// word per (tile, digit) and must be zero on entry; each tile also zeroes its
// own slots of `look_next`, the status array of the following pass.  With a
// payload type V, vin[i] travels with in[i] to the same output slot.
//
// SEG: a segmented pass.  The keys are nseg segments [seg_off[f],
// seg_off[f + 1]), each sorted on its own within its own range; tiles never
// straddle a segment (seg_tiles from k_seg_tiles), digit_base holds
// per-segment digit starts (k_hist_scan with segments), and the look-back of
// a tile stops at its segment's first tile, which publishes an inclusive
// count at once.  Segments already ordered by a key prefix (frames of a
// batch) then need no passes over that prefix.
template <typename K, int RB, int ITEMS, typename V = NoVal, bool SEG = false>
__global__ __launch_bounds__(kSortBlock) void k_onesweep(
    const K *__restrict__ in, K *__restrict__ out, int64_t n_host, const int64_t *d_n, int shift,
    const uint32_t *__restrict__ digit_base, uint32_t *look, uint32_t *look_next,
    uint32_t *tile_ctr, const V *__restrict__ vin = nullptr, V *__restrict__ vout = nullptr,
    const int64_t *__restrict__ seg_off = nullptr, const int64_t *__restrict__ seg_tiles = nullptr,
    int nseg = 0) {
    constexpr bool kHasVal = !std::is_same<V, NoVal>::value;
    constexpr int BLOCK = kSortBlock;
    constexpr int RADIX = 1 << RB;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int DPT = RADIX > BLOCK ? RADIX / BLOCK : 1;  // digits per thread

    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wcnt[WAVES][RADIX];  // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_boff[RADIX];         // block exclusive digit offsets
    __shared__ int64_t s_glob[RADIX];          // global position of LDS slot 0 per digit
    __shared__ uint32_t s_w[WAVES];
    __shared__ K s_keys[TILE];
    __shared__ V s_vals[kHasVal ? TILE : 1];

    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    for (int i = tid; i < WAVES * RADIX; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    int64_t base, n;     // this tile's first key; one past the last key of its range
    uint32_t first = 0;  // first tile of the range the look-back may not leave
    if constexpr (SEG) {
        if ((int64_t)tile >= seg_tiles[nseg]) return;  // uniform across the block
        int lo = 0, len = nseg;  // last segment whose first tile is <= tile
        while (len > 1) {
            const int half = len >> 1;
            lo = seg_tiles[lo + half] <= (int64_t)tile ? lo + half : lo;
            len -= half;
        }
        first = (uint32_t)seg_tiles[lo];
        base = seg_off[lo] + (int64_t)(tile - first) * TILE;
        n = seg_off[lo + 1];
        digit_base += (size_t)lo * RADIX;
    } else {
        n = dev_count(n_host, d_n);
        base = (int64_t)tile * TILE;
        if (base >= n) return;  // uniform across the block
    }

    for (int d = tid; d < RADIX; d += BLOCK) look_next[(size_t)tile * RADIX + d] = 0;

    // Load wave-striped: wave w owns [w*64*ITEMS, (w+1)*64*ITEMS), item i of
    // lane l is element i*64 + l, so (wave, item, lane) order is input order.
    K keys[ITEMS];
    V vals[kHasVal ? ITEMS : 1];
    // a key's digit is recomputed where needed (two instructions) rather
    // than held: registers, not ALU, bound how many tiles a CU keeps in flight
    auto digit = [&](K k) { return (uint32_t)(k >> shift) & (RADIX - 1); };
    const int64_t wbase = base + (int64_t)wave * 64 * ITEMS + lane;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = wbase + i * 64;
        keys[i] = idx < n ? in[idx] : ~K(0);  // padding sorts last, never written
        if constexpr (kHasVal) vals[i] = idx < n ? vin[idx] : V(0);
    }

    // Wave-level multisplit: lanes sharing a digit, found with RB ballots.
    uint32_t rank[ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t di = digit(keys[i]);
        const uint64_t m = match_low_bits<RB>(di);
        uint32_t before = s_wcnt[wave][di];
        uint32_t pre = (uint32_t)__popcll(m & lt);
        rank[i] = before + pre;
        if (pre == 0) s_wcnt[wave][di] = before + (uint32_t)__popcll(m);
    }
    __syncthreads();

    // Per digit: wave offsets and block count.
    uint32_t cnt[DPT];
    uint32_t tsum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        int d = tid * DPT + j;
        uint32_t s = 0;
        if (d < RADIX) {
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                uint32_t c = s_wcnt[w][d];
                s_wcnt[w][d] = s;
                s += c;
            }
            // publish this tile's digit count for the tiles after it
            st_agent(&look[(size_t)tile * RADIX + d], (tile == first ? kFlagInc : kFlagAgg) | s);
        }
        cnt[j] = s;
        tsum += s;
    }
    uint32_t tot;
    uint32_t ex = block_excl_sum<BLOCK>(tsum, s_w, &tot);

    // Decoupled look-back per digit for the count of that digit in all
    // earlier tiles.
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        int d = tid * DPT + j;
        if (d < RADIX) {
            s_boff[d] = ex;
            uint32_t before = 0;
            if (tile > first) {
                // kLookWindow predecessors per round trip: their loads are
                // independent, so a walk over aggregates costs one latency
                // per window, not per tile (the walk ends at the range's
                // first tile, inclusive from the start, before it could
                // count a tile of another segment)
                int64_t t = (int64_t)tile - 1;
                for (;;) {
                    uint32_t st[kLookWindow];
#pragma unroll
                    for (int w = 0; w < kLookWindow; ++w)
                        st[w] = t - w >= 0 ? ld_agent(&look[(size_t)(t - w) * RADIX + d]) : kFlagInc;
                    bool done = false, stall = false;
                    int used = 0;
#pragma unroll
                    for (int w = 0; w < kLookWindow; ++w) {
                        if (done || stall) continue;
                        if ((st[w] & ~kValMask) == 0) {
                            stall = true;  // not published yet: resume here
                            continue;
                        }
                        before += st[w] & kValMask;
                        ++used;
                        done = (st[w] & kFlagInc) != 0;
                    }
                    if (done) break;
                    t -= used;
                    if (stall) __builtin_amdgcn_s_sleep(1);
                }
                st_agent(&look[(size_t)tile * RADIX + d], kFlagInc | (before + cnt[j]));
            }
            s_glob[d] = (int64_t)digit_base[d] + before - ex;
            ex += cnt[j];
        }
    }
    __syncthreads();

    // Stage the tile in LDS in (digit, input order) order.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t di = digit(keys[i]);
        uint32_t pos = s_boff[di] + s_wcnt[wave][di] + rank[i];
        s_keys[pos] = keys[i];
        if constexpr (kHasVal) s_vals[pos] = vals[i];
    }
    __syncthreads();

    // Scatter: consecutive threads write consecutive slots of one bucket.
    // A full tile holds no padding, so every slot is written: straight-line
    // code whose LDS reads the compiler can issue ahead of the stores.
    if (base + TILE <= n) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int j = i * BLOCK + tid;
            const K k = s_keys[j];
            const int64_t g = s_glob[digit(k)] + j;
            out[g] = k;
            if constexpr (kHasVal) vout[g] = s_vals[j];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int j = i * BLOCK + tid;
        K k = s_keys[j];
        int64_t g = s_glob[digit(k)] + j;
        if (g >= 0 && g < n) {
            out[g] = k;
            if constexpr (kHasVal) vout[g] = s_vals[j];
        }
    }
}

// ------------------------------------------------------------------ host
struct SortWs {
    uint32_t *hist = nullptr;   // passes * RADIX (segmented: passes * nseg * RADIX)
    uint32_t *look[2] = {nullptr, nullptr};
    int passes = 0, radix_bits = 8, items = 16;
    int64_t tiles = 0;
    int nseg = 0;
    int64_t *seg_tiles = nullptr;  // segmented: nseg + 1 tile starts
};

// nseg > 0: a segmented sort of nseg segments (histograms per pass and
// segment, up to nseg more tiles, the segment tile table).
inline void sort_carve(Carve &c, SortWs &w, int64_t n, int key_bits, const SortCfg &cfg,
                       int nseg = 0) {
    w.radix_bits = cfg.radix_bits;
    w.items = cfg.items;
    w.passes = sort_passes(key_bits, cfg.radix_bits);
    w.tiles = sort_tiles(n, cfg.items) + nseg;
    w.nseg = nseg;
    const size_t radix = (size_t)1 << cfg.radix_bits;
    w.seg_tiles = nseg > 0 ? c.take<int64_t>((size_t)nseg + 1) : nullptr;
    w.hist = c.take<uint32_t>((size_t)(nseg > 0 ? w.passes * nseg : kMaxPasses) * radix);
    w.look[0] = c.take<uint32_t>((size_t)w.tiles * radix);
    w.look[1] = c.take<uint32_t>((size_t)w.tiles * radix);
}

// Bytes that must be zero before the histogram / first pass.
inline size_t sort_zero_bytes(const SortWs &w) {
    // hist and look[0] are adjacent in the carve order (256-aligned gap ok)
    return (size_t)((char *)w.look[1] - (char *)w.hist);
}

// Items per thread compiled into this library (tiles of 256 x items keys):
// larger tiles write longer runs per bucket and need fewer look-backs, which
// pays on large arrays; smaller ones keep more tiles in flight on small ones.
constexpr int kSortItems[] = {8, 12, 16, 24, 32};

// Digit widths and tile sizes compiled into this library.
inline bool sort_cfg_supported(const SortCfg &c) {
    return (c.radix_bits >= 4 && c.radix_bits <= 11) &&
           (c.items == 8 || c.items == 12 || c.items == 16 || c.items == 24 || c.items == 32);
}

// Autotuned configuration recorded for (key bytes, key bits, n), if any.
bool tuned_sort_cfg(int key_bytes, int key_bits, int64_t n, SortCfg *out);

inline size_t hist_lds_bytes(int passes, int rb) { return (size_t)passes * ((size_t)1 << rb) * 4; }

template <typename K, int RB, int ITEMS>
inline void onesweep_launch(const SortWs &w, const K *src, K *dst, int64_t n_host,
                            const int64_t *d_n, int pass, uint32_t *tile_ctr, hipStream_t s) {
    const size_t radix = (size_t)1 << RB;
    CGA_PROF("onesweep", s);
    k_onesweep<K, RB, ITEMS><<<(unsigned)w.tiles, kSortBlock, 0, s>>>(
        src, dst, n_host, d_n, pass * RB, w.hist + (size_t)pass * radix, w.look[pass & 1],
        w.look[(pass + 1) & 1], tile_ctr + pass);
}

template <typename K, int RB>
inline void onesweep_items(const SortWs &w, const K *src, K *dst, int64_t n_host,
                           const int64_t *d_n, int pass, uint32_t *tile_ctr, hipStream_t s) {
    switch (w.items) {
        case 8: onesweep_launch<K, RB, 8>(w, src, dst, n_host, d_n, pass, tile_ctr, s); break;
        case 12: onesweep_launch<K, RB, 12>(w, src, dst, n_host, d_n, pass, tile_ctr, s); break;
        case 24: onesweep_launch<K, RB, 24>(w, src, dst, n_host, d_n, pass, tile_ctr, s); break;
        case 32: onesweep_launch<K, RB, 32>(w, src, dst, n_host, d_n, pass, tile_ctr, s); break;
        default: onesweep_launch<K, RB, 16>(w, src, dst, n_host, d_n, pass, tile_ctr, s); break;
    }
}

template <typename K, int RB>
inline void sort_launch_rb(const SortWs &w, const K *in, K *out, K *alt0, K *alt1,
                           int64_t n_host, const int64_t *d_n, bool have_hist,
                           uint32_t *tile_ctr, hipStream_t s) {
    if (!have_hist) {
        int64_t blocks = (n_host + kSortBlock * 16 - 1) / (kSortBlock * 16);
        blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
        CGA_PROF("histogram", s);
        k_histogram<K, RB><<<(unsigned)blocks, kSortBlock, hist_lds_bytes(w.passes, RB), s>>>(
            in, n_host, d_n, w.passes, w.hist);
    }
    {
        CGA_PROF("hist_scan", s);
        k_hist_scan<RB><<<(unsigned)w.passes, kSortBlock, 0, s>>>(w.hist);
    }
    // buffer chain: in -> B1 -> ... -> B(P-1) -> out, intermediates alternate
    // so that no pass reads the buffer it writes
    const K *src = in;
    for (int p = 0; p < w.passes; ++p) {
        K *dst;
        if (p == w.passes - 1) dst = out;
        else dst = ((w.passes - 1 - p) & 1) ? alt0 : alt1;
        onesweep_items<K, RB>(w, src, dst, n_host, d_n, p, tile_ctr, s);
        src = dst;
    }
}

// Launch the histogram (unless `have_hist`: already accumulated into w.hist),
// the digit scans and every pass, from `in` to `out` through alt0/alt1.
// When passes == 1 the single pass goes straight from in to out, so in and
// out must differ.  tile_ctr: `passes` zeroed counters.  w.hist and
// w.look[0] must be zero on entry.
template <typename K>
inline void sort_launch(const SortWs &w, const K *in, K *out, K *alt0, K *alt1, int64_t n_host,
                        const int64_t *d_n, bool have_hist, uint32_t *tile_ctr, hipStream_t s) {
    if (w.passes == 0) return;
    switch (w.radix_bits) {
        case 4: sort_launch_rb<K, 4>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 5: sort_launch_rb<K, 5>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 6: sort_launch_rb<K, 6>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 7: sort_launch_rb<K, 7>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 9: sort_launch_rb<K, 9>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 10: sort_launch_rb<K, 10>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        case 11: sort_launch_rb<K, 11>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
        default: sort_launch_rb<K, 8>(w, in, out, alt0, alt1, n_host, d_n, have_hist, tile_ctr, s); break;
    }
}

template <int RB, int ITEMS>
inline void onesweep_seg_launch(const SortWs &w, const uint64_t *src, uint64_t *dst,
                                const int64_t *seg_off, int pass, uint32_t *tile_ctr,
                                hipStream_t s) {
    const size_t radix = (size_t)1 << RB;
    CGA_PROF("onesweep", s);
    k_onesweep<uint64_t, RB, ITEMS, NoVal, true><<<(unsigned)w.tiles, kSortBlock, 0, s>>>(
        src, dst, 0, nullptr, pass * RB, w.hist + (size_t)pass * w.nseg * radix, w.look[pass & 1],
        w.look[(pass + 1) & 1], tile_ctr + pass, nullptr, nullptr, seg_off, w.seg_tiles, w.nseg);
}

template <int RB>
inline void sort_launch_seg_rb(const SortWs &w, const uint64_t *in, uint64_t *out, uint64_t *alt0,
                               uint64_t *alt1, const int64_t *seg_off, uint32_t *tile_ctr,
                               hipStream_t s) {
    {
        CGA_PROF("hist_scan", s);
        k_seg_tiles<1024><<<1, 1024, 0, s>>>(seg_off, w.nseg, (int64_t)kSortBlock * w.items, w.seg_tiles);
        k_hist_scan<RB><<<(unsigned)(w.passes * w.nseg), kSortBlock, 0, s>>>(w.hist, seg_off,
                                                                             w.nseg);
    }
    const uint64_t *src = in;
    for (int p = 0; p < w.passes; ++p) {
        uint64_t *dst = p == w.passes - 1 ? out : (((w.passes - 1 - p) & 1) ? alt0 : alt1);
        switch (w.items) {
            case 8: onesweep_seg_launch<RB, 8>(w, src, dst, seg_off, p, tile_ctr, s); break;
            case 12: onesweep_seg_launch<RB, 12>(w, src, dst, seg_off, p, tile_ctr, s); break;
            case 24: onesweep_seg_launch<RB, 24>(w, src, dst, seg_off, p, tile_ctr, s); break;
            case 32: onesweep_seg_launch<RB, 32>(w, src, dst, seg_off, p, tile_ctr, s); break;
            default: onesweep_seg_launch<RB, 16>(w, src, dst, seg_off, p, tile_ctr, s); break;
        }
        src = dst;
    }
}

// Segmented sort of 64-bit keys (`w` carved with nseg segments): every
// segment [seg_off[f], seg_off[f + 1]) sorted on its own by the low
// passes * radix_bits bits, in place within its range; the histograms
// hist[p][f][digit] already accumulated (the batched encode does that).
// Buffer chain, zeroed state and tile counters as in sort_launch.
inline void sort_launch_seg(const SortWs &w, const uint64_t *in, uint64_t *out, uint64_t *alt0,
                            uint64_t *alt1, const int64_t *seg_off, uint32_t *tile_ctr,
                            hipStream_t s) {
    if (w.passes == 0 || w.nseg < 1) return;
    switch (w.radix_bits) {
        case 4: sort_launch_seg_rb<4>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 5: sort_launch_seg_rb<5>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 6: sort_launch_seg_rb<6>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 7: sort_launch_seg_rb<7>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 9: sort_launch_seg_rb<9>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 10: sort_launch_seg_rb<10>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        case 11: sort_launch_seg_rb<11>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
        default: sort_launch_seg_rb<8>(w, in, out, alt0, alt1, seg_off, tile_ctr, s); break;
    }
}

// Key-value sort (payload uint32_t) with 8-bit digits and 4096-key tiles:
// the same passes as sort_launch, the payload following its key; `w` carved
// with radix_bits 8 and items 16.  Buffer chain as in sort_launch_rb, for the
// keys (in, out, alt0, alt1) and the values (vin, vout, valt0, valt1).
template <typename K>
inline void sort_launch_kv(const SortWs &w, const K *in, K *out, K *alt0, K *alt1,
                           const uint32_t *vin, uint32_t *vout, uint32_t *valt0, uint32_t *valt1,
                           int64_t n_host, const int64_t *d_n, bool have_hist,
                           uint32_t *tile_ctr, hipStream_t s) {
    constexpr int RB = 8, ITEMS = 16;
    if (w.passes == 0) return;
    if (!have_hist) {
        int64_t blocks = (n_host + kSortBlock * 16 - 1) / (kSortBlock * 16);
        blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
        CGA_PROF("histogram", s);
        k_histogram<K, RB><<<(unsigned)blocks, kSortBlock, hist_lds_bytes(w.passes, RB), s>>>(
            in, n_host, d_n, w.passes, w.hist);
    }
    {
        CGA_PROF("hist_scan", s);
        k_hist_scan<RB><<<(unsigned)w.passes, kSortBlock, 0, s>>>(w.hist);
    }
    const K *src = in;
    const uint32_t *vsrc = vin;
    for (int p = 0; p < w.passes; ++p) {
        const bool last = p == w.passes - 1, even = ((w.passes - 1 - p) & 1) != 0;
        K *dst = last ? out : (even ? alt0 : alt1);
        uint32_t *vdst = last ? vout : (even ? valt0 : valt1);
        CGA_PROF("onesweep_kv", s);
        k_onesweep<K, RB, ITEMS, uint32_t><<<(unsigned)w.tiles, kSortBlock, 0, s>>>(
            src, dst, n_host, d_n, p * RB, w.hist + (size_t)p * 256, w.look[p & 1],
            w.look[(p + 1) & 1], tile_ctr + p, vsrc, vdst);
        src = dst;
        vsrc = vdst;
    }
}

}  // namespace cga
