// Run-length compaction of a sorted key sequence: one pass that finds run
// heads (v[i] != v[i-1]) and tails (v[i] != v[i+1]), numbers the runs with a
// block scan plus a decoupled look-back over earlier tiles, and writes one
// value per run and either the run length or the running end offset.
//
// The scanned pair is (heads so far, index of the latest head); the second
// component lets a tail whose head lies in an earlier tile compute its run
// length without a second pass.
#pragma once

#include "cga_common.h"

namespace cga {

constexpr int kRleBlock = 256;
constexpr int kRleItems = 24;
constexpr int kRleTile = kRleBlock * kRleItems;

inline int64_t rle_tiles(int64_t n) { return n <= 0 ? 1 : (n + kRleTile - 1) / kRleTile; }

// status word: [flag:2][heads:31][latest head index + 1:31]
constexpr uint64_t kRleAgg = 1ull << 62;
constexpr uint64_t kRleInc = 2ull << 62;
__device__ __forceinline__ uint64_t rle_pack(uint64_t flag, uint32_t cnt, int32_t last) {
    return flag | ((uint64_t)cnt << 31) | (uint64_t)(uint32_t)(last + 1);
}
__device__ __forceinline__ uint32_t rle_cnt(uint64_t s) { return (uint32_t)((s >> 31) & 0x7FFFFFFFu); }
__device__ __forceinline__ int32_t rle_last(uint64_t s) { return (int32_t)(s & 0x7FFFFFFFu) - 1; }

// v_i = in[i] >> shift.  Per run u (in order): vals[u] = v & out_mask, and
// counts[u] = run length (COUNTS) or ends[u + 1] = one past the run's last
// index with ends[0] = 0 (ENDS).  Either output pointer may be null.
template <typename K, typename OV, bool ENDS>
__global__ __launch_bounds__(kRleBlock) void k_rle(const K *__restrict__ in, int64_t n_host,
                                                   const int64_t *d_n, int shift,
                                                   uint64_t out_mask, OV *__restrict__ vals,
                                                   uint32_t *__restrict__ counts,
                                                   int64_t *__restrict__ ends, int64_t cap,
                                                   int64_t *n_out, uint64_t *status,
                                                   uint32_t *tile_ctr, uint32_t *err) {
    __shared__ uint32_t s_tile;
    // logical slot j lives at j + j/16, so the blocked per-thread reads below
    // (16 consecutive slots per thread) do not all fall in one LDS bank
    __shared__ K s_v[kRleTile + 2 + (kRleTile + 2) / 16 + 1];
#define SV(j) s_v[(j) + ((j) >> 4)]
    __shared__ uint32_t s_wc[kRleBlock / 64];
    __shared__ int32_t s_wl[kRleBlock / 64];
    __shared__ uint32_t s_pc;
    __shared__ int32_t s_pl;

    const int tid = threadIdx.x;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const int64_t n = dev_count(n_host, d_n);
    const int64_t base = (int64_t)tile * kRleTile;
    if (base >= n) return;

    {
        // every load of the tile issued before the first LDS store
        K v[kRleItems];
#pragma unroll
        for (int it = 0; it < kRleItems; ++it) {
            const int64_t i = base + it * kRleBlock + tid;
            v[it] = i < n ? in[i] : K(0);
        }
#pragma unroll
        for (int it = 0; it < kRleItems; ++it) {
            const int j = it * kRleBlock + tid;
            SV(1 + j) = base + j < n ? (K)(v[it] >> shift) : K(0);
        }
    }
    if (tid == 0) SV(0) = base > 0 ? (K)(in[base - 1] >> shift) : K(0);
    if (tid == 1) SV(kRleTile + 1) = base + kRleTile < n ? (K)(in[base + kRleTile] >> shift) : K(0);
    __syncthreads();

    const int j0 = tid * kRleItems;
    uint32_t hc = 0;
    int32_t hl = -1;
#pragma unroll
    for (int it = 0; it < kRleItems; ++it) {
        int j = j0 + it;
        int64_t i = base + j;
        if (i < n && (i == 0 || SV(1 + j) != SV(j))) {
            ++hc;
            hl = (int32_t)i;
        }
    }
    uint32_t tot_c;
    int32_t tot_l;
    uint32_t ex_c = block_excl_sum<kRleBlock>(hc, s_wc, &tot_c);
    int32_t ex_l = block_excl_max<kRleBlock>(hl, (int32_t)-1, s_wl, &tot_l);

    if (tid < 64) {  // wave 0: publish, then look back 64 tiles per round trip
        uint32_t pc = 0;
        int32_t pl = -1;
        if (tile == 0) {
            if (tid == 0) st_agent(&status[tile], rle_pack(kRleInc, tot_c, tot_l));
        } else {
            if (tid == 0) st_agent(&status[tile], rle_pack(kRleAgg, tot_c, tot_l));
            for (int64_t t = tile; ; t -= 64) {
                uint64_t upto;
                const uint64_t st = lookback_window(status, t, 0, &upto);
                const bool use = ((upto ? upto : ~0ull) >> tid) & 1ull;
                // tiles before the first (t - 1 - lane < 0) read as inclusive
                // zeros: count 0, latest head -1
                const bool real = t - 1 - tid >= 0;
                uint32_t c = use && real ? rle_cnt(st) : 0u;
                int32_t l = use && real ? rle_last(st) : -1;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    c += __shfl_xor(c, o, 64);
                    const int32_t lo = __shfl_xor(l, o, 64);
                    l = lo > l ? lo : l;
                }
                pc += c;
                pl = pl > l ? pl : l;
                if (upto) break;
            }
            const int32_t il = pl > tot_l ? pl : tot_l;
            if (tid == 0) st_agent(&status[tile], rle_pack(kRleInc, pc + tot_c, il));
        }
        if (tid == 0) {
            s_pc = pc;
            s_pl = pl;
            if (ENDS && tile == 0 && ends) ends[0] = 0;
        }
    }
    __syncthreads();

    // Outputs go through LDS so that consecutive threads write consecutive
    // slots: first the values of the runs that start in this tile, then the
    // counts (or ends) of the runs that end in it.  Each thread first keeps
    // its items' outputs in registers, as the tile's keys still occupy LDS.
    const uint32_t rc0 = s_pc + ex_c;  // runs that start before this thread's items
    uint32_t rc = rc0;
    int32_t rl = s_pl > ex_l ? s_pl : ex_l;
    K hv[kRleItems];
    uint32_t ev[kRleItems];
    uint32_t hbits = 0, ebits = 0;
#pragma unroll
    for (int it = 0; it < kRleItems; ++it) {
        const int j = j0 + it;
        const int64_t i = base + j;
        hv[it] = K(0);
        ev[it] = 0;
        if (i < n) {
            const K v = SV(1 + j);
            if (i == 0 || v != SV(j)) {
                ++rc;
                rl = (int32_t)i;
                hbits |= 1u << it;
                hv[it] = v;
            }
            if (i == n - 1 || v != SV(2 + j)) {
                ebits |= 1u << it;
                ev[it] = ENDS ? (uint32_t)(i + 1 - base) : (uint32_t)(i + 1 - rl);
                if (i == n - 1 && n_out) *n_out = rc;
            }
        }
    }
    const int64_t tile_end = base + kRleTile < n ? base + kRleTile : n;
    const bool first_head = base == 0 || SV(1) != SV(0);
    const int jl = (int)(tile_end - 1 - base);
    const bool last_end = tile_end == n || SV(1 + jl) != SV(2 + jl);
    __syncthreads();  // every thread has read the tile's keys

    K *st_v = s_v;  // the starts' values, slot = run number - s_pc - 1
#pragma unroll
    for (int it = 0; it < kRleItems; ++it)
        if ((hbits >> it) & 1u) st_v[ex_c + __popc(hbits & ((1u << it) - 1u))] = hv[it];
    __syncthreads();
    for (int j = tid; j < (int)tot_c; j += kRleBlock) {
        const int64_t r = (int64_t)s_pc + j + 1;  // run number, from 1
        if (r <= cap && vals) vals[r - 1] = (OV)((uint64_t)st_v[j] & out_mask);
    }
    if (tid == 0 && (int64_t)s_pc + tot_c > cap) set_err(err, ERR_CAPACITY);
    __syncthreads();

    // the ends' counts (or end offsets within the tile), slot = run number -
    // the run number of the tile's first element
    uint32_t *st_e = (uint32_t *)s_v;
    const uint32_t r_first = s_pc + (first_head ? 1u : 0u);
#pragma unroll
    for (int it = 0; it < kRleItems; ++it)
        if ((ebits >> it) & 1u) st_e[rc0 + __popc(hbits & ((2u << it) - 1u)) - r_first] = ev[it];
    __syncthreads();
    const int ne = (int)tot_c + (first_head ? 0 : 1) - (last_end ? 0 : 1);
    for (int j = tid; j < ne; j += kRleBlock) {
        const int64_t r = (int64_t)r_first + j;
        if (r <= cap) {
            if (ENDS) {
                if (ends) ends[r] = base + st_e[j];
            } else if (counts) {
                counts[r - 1] = st_e[j];
            }
        }
    }
#undef SV
}

}  // namespace cga
