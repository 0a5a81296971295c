// Merge path (Green, McColl & Bader 2012) union of two sorted unique key
// arrays, one window of merged positions per workgroup: the window is merged
// in LDS with A before B on equal keys, the B copy of every key present in
// both is dropped, and survivors are compacted with a decoupled look-back
// over the earlier windows of the same merge.  Shared by the single merge
// and the batched pair merges.
#pragma once

#include "cga_common.h"

namespace cga {

constexpr int kMergeBlock = 256;
constexpr int kMergeItems = 16;
constexpr int kMergeTile = kMergeBlock * kMergeItems;

constexpr uint64_t kMAgg = 1ull << 62;
constexpr uint64_t kMInc = 2ull << 62;
constexpr uint64_t kMVal = (1ull << 62) - 1;

inline int64_t merge_tiles(int64_t total) {
    return total <= 0 ? 1 : (total + kMergeTile - 1) / kMergeTile;
}

// Number of A elements among the first `diag` merged elements, with A
// ordered before B on equal keys.
template <typename K>
__device__ __forceinline__ int64_t merge_path(const K *A, int64_t na, const K *B, int64_t nb,
                                              int64_t diag) {
    int64_t lo = diag > nb ? diag - nb : 0, hi = diag < na ? diag : na;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[diag - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename K>
struct MergeShared {
    K s[kMergeTile + 1];
    uint8_t src[kMergeTile];
    uint32_t w[kMergeBlock / 64];
    int64_t prefix;
};

// Merge window [d0, d1) of A u B (a0 / a1 = A elements before d0 / d1).
// Tile `tile` publishes to status[tile] and looks back no further than
// `seg_first` (the first tile of this merge).  Writes survivors at
// out[prefix...]; the window that ends the merge stores the total count.
template <typename K>
__device__ __forceinline__ void merge_tile(MergeShared<K> &sh, const K *__restrict__ A, int64_t na,
                                           const K *__restrict__ B, int64_t nb, int64_t d0,
                                           int64_t d1, int64_t a0, int64_t a1, K *__restrict__ out,
                                           uint8_t *__restrict__ src_out, int64_t cap,
                                           int64_t *n_out, uint64_t *status, int64_t tile,
                                           int64_t seg_first, uint32_t *err) {
    const int tid = threadIdx.x;
    const int64_t total = na + nb;
    const int64_t b0 = d0 - a0, b1 = d1 - a1;
    const int la = (int)(a1 - a0), lb = (int)(b1 - b0);
    const bool extra = b1 < nb;  // first B element after the window, for provenance
    const int len = la + lb + (extra ? 1 : 0);
    K *s = sh.s;
    {
        // every load of the window issued before the first LDS store
        constexpr int kLoads = (kMergeTile + 1 + kMergeBlock - 1) / kMergeBlock;
        K v[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int j = u * kMergeBlock + tid;
            v[u] = j < len ? (j < la ? A[a0 + j] : B[b0 + (j - la)]) : K(0);
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int j = u * kMergeBlock + tid;
            if (j < len) s[j] = v[u];
        }
    }
    const bool prev_global = a0 > 0;
    const K prev_a_global = prev_global ? A[a0 - 1] : K(0);
    __syncthreads();

    const K *sa = s, *sb = s + la;
    const int lab = la + lb;
    const int dt = tid * kMergeItems < lab ? tid * kMergeItems : lab;
    int at, bt;
    {
        int lo = dt > lb ? dt - lb : 0, hi = dt < la ? dt : la;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (sa[mid] <= sb[dt - 1 - mid]) lo = mid + 1;
            else hi = mid;
        }
        at = lo;
        bt = dt - at;
    }
    bool has_prev = at > 0 || prev_global;
    K prev_a = at > 0 ? sa[at - 1] : prev_a_global;
    const int lb_ext = lb + (extra ? 1 : 0);

    K key[kMergeItems];
    uint8_t srcb[kMergeItems];
    bool keep[kMergeItems];
    uint32_t cnt = 0;
#pragma unroll
    for (int it = 0; it < kMergeItems; ++it) {
        const bool valid = dt + it < lab;
        key[it] = K(0);
        srcb[it] = 0;
        keep[it] = false;
        if (valid) {
            const bool take_a = bt >= lb || (at < la && sa[at] <= sb[bt]);
            if (take_a) {
                K k = sa[at++];
                srcb[it] = (bt < lb_ext && sb[bt] == k) ? 3 : 1;
                prev_a = k;
                has_prev = true;
                key[it] = k;
                keep[it] = true;
            } else {
                K k = sb[bt++];
                key[it] = k;
                srcb[it] = 2;
                keep[it] = !(has_prev && prev_a == k);
            }
            cnt += keep[it] ? 1u : 0u;
        }
    }
    uint32_t tot;
    uint32_t ex = block_excl_sum<kMergeBlock>(cnt, sh.w, &tot);

    if (tid < 64) {  // wave 0: publish, look back over earlier windows of this merge
        uint64_t pre = 0;
        if (tile == seg_first) {
            if (tid == 0) st_agent(&status[tile], kMInc | (uint64_t)tot);
        } else {
            if (tid == 0) st_agent(&status[tile], kMAgg | (uint64_t)tot);
            pre = lookback_sum62(status, tile, seg_first);
            if (tid == 0) st_agent(&status[tile], kMInc | (pre + tot));
        }
        if (tid == 0) {
            sh.prefix = (int64_t)pre;
            if (d1 == total && n_out) *n_out = (int64_t)pre + tot;
        }
    }
    // stage survivors in LDS (the merge reads of s finished at the scan's barriers)
    uint32_t o = ex;
#pragma unroll
    for (int it = 0; it < kMergeItems; ++it)
        if (keep[it]) {
            s[o] = key[it];
            sh.src[o] = srcb[it];
            ++o;
        }
    __syncthreads();
    const int64_t pre = sh.prefix;
    bool over = false;
    for (int j = tid; j < (int)tot; j += kMergeBlock) {
        int64_t g = pre + j;
        if (g < cap) {
            out[g] = s[j];
            if (src_out) src_out[g] = sh.src[j];
        } else {
            over = true;
        }
    }
    if (over) set_err(err, ERR_CAPACITY);
    __syncthreads();  // LDS is reused by the next window of a persistent loop
}

}  // namespace cga
