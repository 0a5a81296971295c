// Orthogonal projection, Eq. (3) with m_x = m_y = 1 (Section V-B): re-key
// every voxel to the 2-D pixel left after dropping one axis, sort the pixel
// keys, and collapse equal pixels with their voxel counts.  In LINEAR order
// dropping z is monotone (key >> depth), so that case skips the sort.
#include "cga_common.h"
#include "cga_rle.h"
#include "cga_sort.h"

namespace cga {

SortCfg default_sort_cfg(bool wide, int64_t n, int key_bits);

template <typename K, typename K2, int RB>
__global__ __launch_bounds__(256) void k_rekey(const K *__restrict__ in, int64_t n_host,
                                               const int64_t *d_n, uint32_t depth, int linear,
                                               int drop, K2 *__restrict__ out, int passes,
                                               uint32_t *hist) {
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_h[];
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const int64_t n = dev_count(n_host, d_n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        Vox v = dec3(in[i], depth, linear != 0);
        uint32_t u = drop == 0 ? v.y : v.x;
        uint32_t w = drop == 2 ? v.y : v.z;
        K2 k2 = linear ? (K2)(((uint64_t)u << depth) | w) : (K2)((spread2(u) << 1) | spread2(w));
        out[i] = k2;
        hist_add_coherent<RB>(s_h, k2, passes);
    }
    __syncthreads();
    hist_flush<RB>(s_h, hist, passes);
}

template <typename K, typename K2, int RB>
static void rekey_launch(const K *in, int64_t n, const int64_t *d_n, const cga_grid *g, int drop,
                         K2 *out, int passes, uint32_t *hist, hipStream_t s) {
    int64_t blocks = (n + 256 * 8 - 1) / (256 * 8);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    CGA_PROF("rekey", s);
    k_rekey<K, K2, RB><<<(unsigned)blocks, 256, hist_lds_bytes(passes, RB), s>>>(
        in, n, d_n, g->depth, g->key_mode == CGA_KEY_LINEAR, drop, out, passes, hist);
}

template <typename K, typename K2>
static void rekey_dispatch(int rb, const K *in, int64_t n, const int64_t *d_n, const cga_grid *g,
                           int drop, K2 *out, int passes, uint32_t *hist, hipStream_t s) {
    switch (rb) {
        case 4: rekey_launch<K, K2, 4>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 5: rekey_launch<K, K2, 5>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 6: rekey_launch<K, K2, 6>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 7: rekey_launch<K, K2, 7>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 9: rekey_launch<K, K2, 9>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 10: rekey_launch<K, K2, 10>(in, n, d_n, g, drop, out, passes, hist, s); break;
        case 11: rekey_launch<K, K2, 11>(in, n, d_n, g, drop, out, passes, hist, s); break;
        default: rekey_launch<K, K2, 8>(in, n, d_n, g, drop, out, passes, hist, s); break;
    }
}

struct ProjLayout {
    Control *ctl;
    SortWs sort;
    uint64_t *rle_status;
    void *buf_a, *buf_b;
    size_t bytes;
};

static ProjLayout proj_layout(void *ws, const cga_grid *g, int64_t n, const SortCfg &cfg) {
    ProjLayout L;
    Carve c(ws);
    const size_t kb = wide_keys2(g->depth) ? 8 : 4;
    L.ctl = c.take<Control>(1);
    sort_carve(c, L.sort, n, 2 * (int)g->depth, cfg);
    L.rle_status = c.take<uint64_t>((size_t)rle_tiles(n));
    L.buf_a = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    L.buf_b = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    L.bytes = c.size();
    return L;
}

template <typename K, typename K2>
static void project_enqueue(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                            int drop, K2 *out, uint32_t *counts, int64_t cap, int64_t *n_out,
                            const ProjLayout &L, hipStream_t s) {
    const uint32_t d = g->depth;
    if (g->key_mode == CGA_KEY_LINEAR && drop == 2) {
        // (x<<2d | y<<d | z) >> d = x<<d | y: already ascending, just collapse
        CGA_PROF("rle", s);
        k_rle<K, K2, false><<<(unsigned)rle_tiles(n), kRleBlock, 0, s>>>(
            keys, n, d_n, (int)d, ~0ull, out, counts, nullptr, cap, n_out, L.rle_status,
            &L.ctl->tile_ctr[kMaxPasses], &L.ctl->err);
        return;
    }
    const SortWs &w = L.sort;
    K2 *a = (K2 *)L.buf_a, *b = (K2 *)L.buf_b;
    rekey_dispatch<K, K2>(w.radix_bits, keys, n, d_n, g, drop, a, w.passes, w.hist, s);
    K2 *fin = (w.passes & 1) ? b : a;
    K2 *other = (w.passes & 1) ? a : b;
    sort_launch<K2>(w, a, fin, other, fin, n, d_n, true, L.ctl->tile_ctr, s);
    CGA_PROF("rle", s);
    k_rle<K2, K2, false><<<(unsigned)rle_tiles(n), kRleBlock, 0, s>>>(
        fin, n, d_n, 0, ~0ull, out, counts, nullptr, cap, n_out, L.rle_status,
        &L.ctl->tile_ctr[kMaxPasses], &L.ctl->err);
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_project_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    size_t m = 0;
    for (int rb = 4; rb <= 11; ++rb)
        for (int items : kSortItems) {
            SortCfg c;
            c.radix_bits = rb;
            c.items = items;
            size_t b = proj_layout(nullptr, g, n, c).bytes;
            m = b > m ? b : m;
        }
    return m;
}

int cga_project(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                int drop_axis, void *d_out2d, uint32_t *d_counts, int64_t cap, int64_t *d_n_out,
                int64_t *n_out_host, void *d_ws, size_t ws_bytes, const cga_tune *tune,
                cga_stream stream) {
    if (!grid_valid(g) || n < 0 || cap < 0 || !d_ws) return CGA_EINVAL;
    if (drop_axis < 0 || drop_axis > 2) return CGA_EINVAL;
    if (n > 0 && (!d_keys || !d_out2d)) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    const bool wide2 = wide_keys2(g->depth);
    SortCfg cfg = default_sort_cfg(wide2, n, 2 * (int)g->depth);
    if (!tune) tuned_sort_cfg(wide2 ? 8 : 4, 2 * (int)g->depth, n, &cfg);
    if (tune) {
        cfg.radix_bits = (int)tune->radix_bits;
        cfg.items = (int)tune->tile_items;
        if (!sort_cfg_supported(cfg)) return CGA_EINVAL;
    }
    ProjLayout L = proj_layout(d_ws, g, n, cfg);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int64_t *cnt_out = d_n_out ? d_n_out : &L.ctl->count;
    CGA_TRY(launch_begin(L.ctl, L.sort.hist, sort_zero_bytes(L.sort), L.rle_status,
                         (size_t)rle_tiles(n) * 8, cnt_out, s));
    if (n > 0) {
        if (!wide_keys(g->depth))
            project_enqueue<uint32_t, uint32_t>(g, (const uint32_t *)d_keys, n, d_n, drop_axis,
                                                (uint32_t *)d_out2d, d_counts, cap, cnt_out, L, s);
        else if (!wide2)
            project_enqueue<uint64_t, uint32_t>(g, (const uint64_t *)d_keys, n, d_n, drop_axis,
                                                (uint32_t *)d_out2d, d_counts, cap, cnt_out, L, s);
        else
            project_enqueue<uint64_t, uint64_t>(g, (const uint64_t *)d_keys, n, d_n, drop_axis,
                                                (uint64_t *)d_out2d, d_counts, cap, cnt_out, L, s);
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
