// Merge, Eq. (1): union of two sorted unique key arrays by merge path
// (Green, McColl & Bader 2012).  Each workgroup owns a fixed-size window of
// merged positions, finds where it starts in A and B from a precomputed
// partition, merges in LDS (A before B on equal keys), drops the B copy of
// every key present in both, and compacts its survivors with a decoupled
// look-back over earlier windows.
#include "cga_common.h"
#include "cga_merge.h"

#include <mutex>

namespace cga {

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
    __shared__ MergeShared<K> sh;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const int64_t na = dev_count(na_host, d_na), nb = dev_count(nb_host, d_nb);
    const int64_t total = na + nb;
    const int64_t d0 = (int64_t)tile * kMergeTile;
    if (d0 >= total) return;
    const int64_t d1 = d0 + kMergeTile < total ? d0 + kMergeTile : total;
    merge_tile<K>(sh, A, na, B, nb, d0, d1, part[tile], part[tile + 1], out, src_out, cap, n_out,
                  status, tile, 0, err);
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

// The merge body shared by cga_merge and cga_merge_noalloc; d_ws is the
// workspace device address (a caller buffer or the static scratch array).
static int merge_call(const cga_grid *g, const void *d_a, int64_t na, const int64_t *d_na,
                      const void *d_b, int64_t nb, const int64_t *d_nb, void *d_out, uint8_t *d_src,
                      int64_t cap, int64_t *d_n_out, int64_t *n_out_host, void *d_ws,
                      size_t ws_bytes, cga_stream stream) {
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

static bool merge_args_valid(const cga_grid *g, const void *d_a, int64_t na, const void *d_b,
                             int64_t nb, const void *d_out, int64_t cap) {
    if (!grid_valid(g) || na < 0 || nb < 0 || cap < 0) return false;
    return !((na > 0 && !d_a) || (nb > 0 && !d_b) || (na + nb > 0 && !d_out));
}

// Workspace of cga_merge_noalloc: a file-scope device array, one copy per
// GPU, sized for CGA_MERGE_NOALLOC_MAX_KEYS merged positions (a control
// block, then one partition and one look-back word per 2048-key window).
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr size_t kMergeScratchBytes = (size_t)2 << 20 | 4096;
static __device__ __align__(256) char scratch[kMergeScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int merge_scratch(void **out) {
    int dev = -1;
    CGA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return CGA_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        CGA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return CGA_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CGA_OK;
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
    if (!merge_args_valid(g, d_a, na, d_b, nb, d_out, cap) || !d_ws) return CGA_EINVAL;
    if (na + nb >= ((int64_t)1 << 31)) return CGA_EUNSUPPORTED;
    return merge_call(g, d_a, na, d_na, d_b, nb, d_nb, d_out, d_src, cap, d_n_out, n_out_host, d_ws,
                      ws_bytes, stream);
}

int cga_merge_noalloc(const cga_grid *g, const void *d_a, int64_t na, const int64_t *d_na,
                      const void *d_b, int64_t nb, const int64_t *d_nb, void *d_out,
                      uint8_t *d_src, int64_t cap, int64_t *d_n_out, int64_t *n_out_host,
                      cga_stream stream) {
    if (!merge_args_valid(g, d_a, na, d_b, nb, d_out, cap)) return CGA_EINVAL;
    if (na > CGA_MERGE_NOALLOC_MAX_KEYS || nb > CGA_MERGE_NOALLOC_MAX_KEYS - na)
        return CGA_EWORKSPACE;
    static_assert(CGA_MERGE_NOALLOC_MAX_KEYS % kMergeTile == 0, "whole windows");
    if (merge_layout(nullptr, CGA_MERGE_NOALLOC_MAX_KEYS, 0).bytes > kMergeScratchBytes)
        return CGA_EWORKSPACE;  // unreachable: the array holds the largest layout
    void *ws = nullptr;
    CGA_TRY(merge_scratch(&ws));
    return merge_call(g, d_a, na, d_na, d_b, nb, d_nb, d_out, d_src, cap, d_n_out, n_out_host, ws,
                      kMergeScratchBytes, stream);
}

}  // extern "C"
