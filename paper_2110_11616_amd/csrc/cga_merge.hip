// Merge, Eq. (1): union of two sorted unique key arrays by merge path
// (Green, McColl & Bader 2012).  Each workgroup owns a fixed-size window of
// merged positions, finds where it starts in A and B from a precomputed
// partition, merges in LDS (A before B on equal keys), drops the B copy of
// every key present in both, and compacts its survivors with a decoupled
// look-back over earlier windows.
#include "cga_common.h"

namespace cga {

constexpr int kMergeBlock = 256;
constexpr int kMergeItems = 8;
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
__global__ void k_merge_partition(const K *A, int64_t na_host, const int64_t *d_na, const K *B,
                                  int64_t nb_host, const int64_t *d_nb, int64_t *part,
                                  int64_t nparts) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nparts) return;
    const int64_t na = dev_count(na_host, d_na), nb = dev_count(nb_host, d_nb);
    int64_t diag = t * kMergeTile;
    diag = diag < na + nb ? diag : na + nb;
    part[t] = merge_path(A, na, B, nb, diag);
}

template <typename K>
__global__ __launch_bounds__(kMergeBlock) void k_merge(
    const K *__restrict__ A, int64_t na_host, const int64_t *d_na, const K *__restrict__ B,
    int64_t nb_host, const int64_t *d_nb, const int64_t *__restrict__ part, K *__restrict__ out,
    uint8_t *__restrict__ src_out, int64_t cap, int64_t *n_out, uint64_t *status,
    uint32_t *tile_ctr, uint32_t *err) {
    __shared__ uint32_t s_tile;
    __shared__ K s[kMergeTile + 1];
    __shared__ uint8_t s_src[kMergeTile];
    __shared__ uint32_t s_w[kMergeBlock / 64];
    __shared__ int64_t s_prefix;

    const int tid = threadIdx.x;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const int64_t na = dev_count(na_host, d_na), nb = dev_count(nb_host, d_nb);
    const int64_t total = na + nb;
    const int64_t d0 = (int64_t)tile * kMergeTile;
    if (d0 >= total) return;
    const int64_t d1 = d0 + kMergeTile < total ? d0 + kMergeTile : total;
    const int64_t a0 = part[tile], a1 = part[tile + 1];
    const int64_t b0 = d0 - a0, b1 = d1 - a1;
    const int la = (int)(a1 - a0), lb = (int)(b1 - b0);
    const bool extra = b1 < nb;  // first B element after the window, for provenance
    const int len = la + lb + (extra ? 1 : 0);
    for (int j = tid; j < len; j += kMergeBlock)
        s[j] = j < la ? A[a0 + j] : B[b0 + (j - la)];
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
        const bool valid = dt + it < lab && tid * kMergeItems + it < lab;
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
    uint32_t ex = block_excl_sum<kMergeBlock>(cnt, s_w, &tot);

    if (tid == 0) {
        uint64_t pre = 0;
        if (tile == 0) {
            st_agent(&status[tile], kMInc | (uint64_t)tot);
        } else {
            st_agent(&status[tile], kMAgg | (uint64_t)tot);
            int64_t t = (int64_t)tile - 1;
            for (;;) {
                uint64_t st = ld_agent(&status[t]);
                if ((st >> 62) == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                pre += st & kMVal;
                if (st & kMInc) break;
                --t;
            }
            st_agent(&status[tile], kMInc | (pre + tot));
        }
        s_prefix = (int64_t)pre;
        if (d1 == total && n_out) *n_out = (int64_t)pre + tot;
    }
    // stage survivors in LDS (the merge reads of s finished at the scan's barriers)
    uint32_t o = ex;
#pragma unroll
    for (int it = 0; it < kMergeItems; ++it)
        if (keep[it]) {
            s[o] = key[it];
            s_src[o] = srcb[it];
            ++o;
        }
    __syncthreads();
    const int64_t pre = s_prefix;
    bool over = false;
    for (int j = tid; j < (int)tot; j += kMergeBlock) {
        int64_t g = pre + j;
        if (g < cap) {
            out[g] = s[j];
            if (src_out) src_out[g] = s_src[j];
        } else {
            over = true;
        }
    }
    if (over) set_err(err, ERR_CAPACITY);
}

struct MergeLayout {
    Control *ctl;
    int64_t *part;
    uint64_t *status;
    size_t bytes;
};

static MergeLayout merge_layout(void *ws, int64_t na, int64_t nb) {
    MergeLayout L;
    Carve c(ws);
    const int64_t tiles = merge_tiles(na + nb);
    L.ctl = c.take<Control>(1);
    L.part = c.take<int64_t>((size_t)tiles + 1);
    L.status = c.take<uint64_t>((size_t)tiles);
    L.bytes = c.size();
    return L;
}

template <typename K>
static void merge_enqueue(const K *a, int64_t na, const int64_t *d_na, const K *b, int64_t nb,
                          const int64_t *d_nb, K *out, uint8_t *src, int64_t cap, int64_t *n_out,
                          const MergeLayout &L, hipStream_t s) {
    const int64_t tiles = merge_tiles(na + nb);
    const int64_t nparts = tiles + 1;
    {
    CGA_PROF("merge_partition", s);
    k_merge_partition<K><<<(unsigned)((nparts + 255) / 256), 256, 0, s>>>(a, na, d_na, b, nb, d_nb,
                                                                          L.part, nparts);
    }
    CGA_PROF("merge", s);
    k_merge<K><<<(unsigned)tiles, kMergeBlock, 0, s>>>(a, na, d_na, b, nb, d_nb, L.part, out, src,
                                                       cap, n_out, L.status, &L.ctl->tile_ctr[0],
                                                       &L.ctl->err);
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_merge_workspace_bytes(const cga_grid *g, int64_t na, int64_t nb) {
    if (!grid_valid(g) || na < 0 || nb < 0) return 0;
    return merge_layout(nullptr, na, nb).bytes;
}

int cga_merge(const cga_grid *g, const void *d_a, int64_t na, const int64_t *d_na, const void *d_b,
              int64_t nb, const int64_t *d_nb, void *d_out, uint8_t *d_src, int64_t cap,
              int64_t *d_n_out, int64_t *n_out_host, void *d_ws, size_t ws_bytes,
              cga_stream stream) {
    if (!grid_valid(g) || na < 0 || nb < 0 || cap < 0 || !d_ws) return CGA_EINVAL;
    if ((na > 0 && !d_a) || (nb > 0 && !d_b) || (na + nb > 0 && !d_out)) return CGA_EINVAL;
    if (na + nb >= ((int64_t)1 << 31)) return CGA_EUNSUPPORTED;
    MergeLayout L = merge_layout(d_ws, na, nb);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int64_t *cnt_out = d_n_out ? d_n_out : &L.ctl->count;
    CGA_TRY(launch_begin(L.ctl, L.status, (size_t)merge_tiles(na + nb) * 8, nullptr, 0, cnt_out, s));
    if (na + nb > 0) {
        if (wide_keys(g->depth))
            merge_enqueue<uint64_t>((const uint64_t *)d_a, na, d_na, (const uint64_t *)d_b, nb, d_nb,
                                    (uint64_t *)d_out, d_src, cap, cnt_out, L, s);
        else
            merge_enqueue<uint32_t>((const uint32_t *)d_a, na, d_na, (const uint32_t *)d_b, nb, d_nb,
                                    (uint32_t *)d_out, d_src, cap, cnt_out, L, s);
        CGA_HIP(hipGetLastError());
    }
    if (n_out_host) {
        int st = finish_sync(L.ctl, s);
        CGA_HIP(hipMemcpyAsync(n_out_host, cnt_out, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CGA_HIP(hipStreamSynchronize(s));
        return st;
    }
    return CGA_OK;
}

}  // extern "C"
