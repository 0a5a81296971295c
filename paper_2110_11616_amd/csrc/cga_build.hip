// CGA construction (Section V): quantize + encode, radix sort, run-length
// compaction; plus the paper's five coordinate arrays and the shared host
// helpers of the library.
#include <cmath>

#include "cga_common.h"
#include "cga_rle.h"
#include "cga_encode.h"
#include "cga_sort.h"

namespace cga {

thread_local int g_last_hip_error = 0;

bool grid_valid(const cga_grid *g) {
    if (!g) return false;
    if (g->depth < 1 || g->depth > 21) return false;
    if (g->key_mode != CGA_KEY_MORTON && g->key_mode != CGA_KEY_LINEAR) return false;
    if (!std::isfinite(g->scale) || !(g->scale > 0.0f)) return false;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g->origin[a])) return false;
    return true;
}

int status_from_bits(uint32_t bits) {
    if (bits & ERR_NONFINITE) return CGA_ENONFINITE;
    if (bits & ERR_CAPACITY) return CGA_ECAPACITY;
    if (bits & ERR_MISMATCH) return CGA_EMISMATCH;
    return CGA_OK;
}

struct ZeroPtrs {
    int64_t *p[4];
};

// Call prologue: zero the control block, up to two workspace regions and up
// to four int64 outputs.  A kernel rather than memset nodes, so that a
// captured graph replays it faithfully.
__global__ void k_begin(uint32_t *ctl, uint4 *z0, size_t z0_n, uint4 *z1, size_t z1_n,
                        ZeroPtrs zp) {
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    if (tid < kControlBytes / 4) ctl[tid] = 0;
    for (size_t i = tid; i < z0_n; i += stride) z0[i] = make_uint4(0, 0, 0, 0);
    for (size_t i = tid; i < z1_n; i += stride) z1[i] = make_uint4(0, 0, 0, 0);
    if (tid < 4 && zp.p[tid]) *zp.p[tid] = 0;
}

int launch_begin(Control *ctl, void *z0, size_t z0_bytes, void *z1, size_t z1_bytes,
                 int64_t *d_n_out, hipStream_t s, int64_t *zero2, int64_t *zero3,
                 int64_t *zero4) {
    size_t n0 = z0 ? (z0_bytes + 15) / 16 : 0, n1 = z1 ? (z1_bytes + 15) / 16 : 0;
    size_t m = n0 > n1 ? n0 : n1;
    size_t blocks = (m + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    ZeroPtrs zp{{d_n_out, zero2, zero3, zero4}};
    CGA_PROF("begin", s);
    k_begin<<<(unsigned)blocks, 256, 0, s>>>((uint32_t *)ctl, (uint4 *)z0, n0, (uint4 *)z1, n1, zp);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

int finish_sync(const Control *ctl, hipStream_t s) {
    uint32_t bits = 0;
    CGA_HIP(hipMemcpyAsync(&bits, &ctl->err, sizeof bits, hipMemcpyDeviceToHost, s));
    CGA_HIP(hipStreamSynchronize(s));
    return status_from_bits(bits);
}

// Host copy of a device count, after the stream has drained.
static int read_count(const int64_t *d, int64_t *h, hipStream_t s) {
    CGA_HIP(hipMemcpyAsync(h, d, sizeof *h, hipMemcpyDeviceToHost, s));
    CGA_HIP(hipStreamSynchronize(s));
    return CGA_OK;
}

// Default tuning; the autotuner cache may override it per (key width, key
// bits, n).  Digits: the fewest passes that 8-bit digits allow, each as
// narrow as that pass count permits (42-bit keys: six 7-bit passes; 36-bit:
// five 8-bit) -- fewer buckets per tile mean longer bucket runs in the
// scatter and fewer look-back words.  Tiles: 256 threads x 16 keys below 2^22
// keys (enough tiles to fill the chip), else x 24 (64-bit keys) or x 32
// (32-bit keys).  These are the autotuner's picks on MI355X for 10M 64-bit
// keys of 42 bits and 20M 32-bit keys of 28 bits.
SortCfg default_sort_cfg(bool wide, int64_t n, int key_bits) {
    SortCfg c;
    const int bits = key_bits > 0 ? key_bits : (wide ? 64 : 32);
    const int passes = (bits + 7) / 8;
    c.radix_bits = (bits + passes - 1) / passes;
    if (c.radix_bits < 4) c.radix_bits = 4;
    c.items = n < ((int64_t)1 << 22) ? 16 : (wide ? 24 : 32);
    return c;
}

static int pick_cfg(const cga_tune *t, bool wide, int64_t n, SortCfg *out, int key_bits = 0) {
    SortCfg c = default_sort_cfg(wide, n, key_bits);
    if (!t && key_bits > 0) tuned_sort_cfg(wide ? 8 : 4, key_bits, n, &c);
    if (t) {
        c.radix_bits = (int)t->radix_bits;
        c.items = (int)t->tile_items;
        if (!sort_cfg_supported(c)) return CGA_EINVAL;
    }
    *out = c;
    return CGA_OK;
}

// ------------------------------------------------------------- build
struct BuildLayout {
    Control *ctl;
    SortWs sort;
    uint64_t *rle_status;
    void *buf_a, *buf_b;
    size_t bytes;
};

static BuildLayout build_layout(void *ws, const cga_grid *g, int64_t n, const SortCfg &cfg) {
    BuildLayout L;
    Carve c(ws);
    const size_t kb = wide_keys(g->depth) ? 8 : 4;
    L.ctl = c.take<Control>(1);
    sort_carve(c, L.sort, n, 3 * (int)g->depth, cfg);
    L.rle_status = c.take<uint64_t>((size_t)rle_tiles(n));
    L.buf_a = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    L.buf_b = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    L.bytes = c.size();
    return L;
}

// Buffer chain of a P-pass sort that starts in `a` and ping-pongs a <-> b:
// it ends in b when P is odd, in a when P is even.
template <typename K>
static K *sort_chain(const SortWs &w, K *a, K *b, int64_t n, const int64_t *d_n, bool have_hist,
                     uint32_t *tile_ctr, hipStream_t s) {
    if (w.passes == 0) return a;
    K *fin = (w.passes & 1) ? b : a;
    K *other = (w.passes & 1) ? a : b;
    sort_launch<K>(w, a, fin, other, fin, n, d_n, have_hist, tile_ctr, s);
    return fin;
}

template <typename K>
static void build_enqueue(const cga_grid *g, const float *xyz, int64_t n, K *keys,
                          uint32_t *counts, int64_t cap, int64_t *n_out, const BuildLayout &L,
                          hipStream_t s) {
    K *a = (K *)L.buf_a, *b = (K *)L.buf_b;
    const SortWs &w = L.sort;
    encode_dispatch<K>(g, xyz, n, a, w.radix_bits, w.passes, w.hist, &L.ctl->err, s);
    K *fin = sort_chain<K>(w, a, b, n, nullptr, true, L.ctl->tile_ctr, s);
    CGA_PROF("rle", s);
    k_rle<K, K, false><<<(unsigned)rle_tiles(n), kRleBlock, 0, s>>>(
        fin, n, nullptr, 0, ~0ull, keys, counts, nullptr, cap, n_out, L.rle_status,
        &L.ctl->tile_ctr[kMaxPasses], &L.ctl->err);
}

// Largest workspace any compiled tuning needs.
template <typename F>
static size_t max_over_cfgs(F layout_bytes) {
    size_t m = 0;
    for (int rb = 4; rb <= 11; ++rb)
        for (int items : kSortItems) {
            SortCfg c;
            c.radix_bits = rb;
            c.items = items;
            size_t b = layout_bytes(c);
            m = b > m ? b : m;
        }
    return m;
}

// Low `bits` bits of each of the first n values, as uint32.
template <typename K>
__global__ void k_low_bits(const K *__restrict__ in, int64_t n_host, const int64_t *d_n,
                           uint64_t mask, uint32_t *__restrict__ out) {
    const int64_t n = dev_count(n_host, d_n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)((uint64_t)in[i] & mask);
}

struct ArraysLayout {
    Control *ctl;
    uint64_t *st_xy, *st_x;
    void *xy;
    size_t bytes;
};

static ArraysLayout arrays_layout(void *ws, const cga_grid *g, int64_t n) {
    ArraysLayout L;
    Carve c(ws);
    L.ctl = c.take<Control>(1);
    L.st_xy = c.take<uint64_t>((size_t)rle_tiles(n));
    L.st_x = c.take<uint64_t>((size_t)rle_tiles(n));
    L.xy = c.take<char>((size_t)(n > 0 ? n : 1) * (wide_keys(g->depth) ? 8 : 4));
    L.bytes = c.size();
    return L;
}

// Paper arrays from LINEAR keys x<<2d | y<<d | z: the (x, y) runs give
// Y_index and Y_pointer, the x runs over those give X_index and X_pointer.
template <typename K>
static void arrays_enqueue(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                           uint32_t *xi, int64_t *xp, uint32_t *yi, int64_t *yp, uint32_t *zi,
                           int64_t *nx, int64_t *nxy, const ArraysLayout &L, hipStream_t s) {
    const int d = (int)g->depth;
    const uint64_t m = (1ull << d) - 1;
    K *xy = (K *)L.xy;
    const unsigned tiles = (unsigned)rle_tiles(n);
    CGA_PROF("arrays", s);
    k_rle<K, K, true><<<tiles, kRleBlock, 0, s>>>(keys, n, d_n, d, ~0ull, xy, nullptr, yp, n, nxy,
                                                   L.st_xy, &L.ctl->tile_ctr[0], &L.ctl->err);
    k_rle<K, uint32_t, true><<<tiles, kRleBlock, 0, s>>>(xy, n, nxy, d, m, xi, nullptr, xp, n, nx,
                                                         L.st_x, &L.ctl->tile_ctr[1], &L.ctl->err);
    int64_t blocks = (n + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    k_low_bits<K><<<(unsigned)blocks, 256, 0, s>>>(keys, n, d_n, m, zi);
    k_low_bits<K><<<(unsigned)blocks, 256, 0, s>>>(xy, n, nxy, m, yi);
}

}  // namespace cga

using namespace cga;

extern "C" {

const char *cga_strerror(int st) {
    switch (st) {
        case CGA_OK: return "ok";
        case CGA_EINVAL: return "invalid argument";
        case CGA_ECAPACITY: return "output exceeds capacity";
        case CGA_EMISMATCH: return "operand mismatch";
        case CGA_ENONFINITE: return "non-finite coordinate";
        case CGA_EHIP: return "HIP runtime error";
        case CGA_EWORKSPACE: return "workspace too small";
        case CGA_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

int cga_last_hip_error(void) { return g_last_hip_error; }

size_t cga_key_bytes(const cga_grid *g) {
    if (!grid_valid(g)) return 0;
    return wide_keys(g->depth) ? 8 : 4;
}

size_t cga_key2_bytes(const cga_grid *g) {
    if (!grid_valid(g)) return 0;
    return wide_keys2(g->depth) ? 8 : 4;
}

int cga_ws_status(const void *d_ws, cga_stream stream) {
    if (!d_ws) return CGA_EINVAL;
    return finish_sync((const Control *)d_ws, (hipStream_t)stream);
}

size_t cga_build_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    return max_over_cfgs([&](const SortCfg &c) { return build_layout(nullptr, g, n, c).bytes; });
}

int cga_build(const cga_grid *g, const float *d_xyz, int64_t n, void *d_keys, uint32_t *d_counts,
              int64_t cap, int64_t *d_n_out, int64_t *n_out_host, void *d_ws, size_t ws_bytes,
              const cga_tune *tune, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || cap < 0 || !d_ws) return CGA_EINVAL;
    if (n > 0 && (!d_xyz || !d_keys)) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    const bool wide = wide_keys(g->depth);
    SortCfg cfg;
    CGA_TRY(pick_cfg(tune, wide, n, &cfg, 3 * (int)g->depth));
    BuildLayout L = build_layout(d_ws, g, n, cfg);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int64_t *cnt_out = d_n_out ? d_n_out : &L.ctl->count;
    CGA_TRY(launch_begin(L.ctl, L.sort.hist, sort_zero_bytes(L.sort), L.rle_status,
                         (size_t)rle_tiles(n) * 8, cnt_out, s));
    if (n > 0) {
        if (wide)
            build_enqueue<uint64_t>(g, d_xyz, n, (uint64_t *)d_keys, d_counts, cap, cnt_out, L, s);
        else
            build_enqueue<uint32_t>(g, d_xyz, n, (uint32_t *)d_keys, d_counts, cap, cnt_out, L, s);
        CGA_HIP(hipGetLastError());
    }
    if (n_out_host) {
        int st = finish_sync(L.ctl, s);
        CGA_TRY(read_count(cnt_out, n_out_host, s));
        return st;
    }
    return CGA_OK;
}

int cga_encode_keys(const cga_grid *g, const float *d_xyz, int64_t n, void *d_keys, void *d_ws,
                    size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || !d_ws) return CGA_EINVAL;
    if (n > 0 && (!d_xyz || !d_keys)) return CGA_EINVAL;
    if (ws_bytes < kControlBytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Control *ctl = (Control *)d_ws;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (n > 0) {
        if (wide_keys(g->depth))
            encode_dispatch<uint64_t>(g, d_xyz, n, (uint64_t *)d_keys, 8, 0, nullptr, &ctl->err, s);
        else
            encode_dispatch<uint32_t>(g, d_xyz, n, (uint32_t *)d_keys, 8, 0, nullptr, &ctl->err, s);
        CGA_HIP(hipGetLastError());
    }
    return CGA_OK;
}

// ---------------------------------------------------------------- sort
static size_t sort_api_layout(void *ws, const cga_grid *g, int64_t n, const SortCfg &cfg,
                              Control **ctl, SortWs *w, void **a, void **b) {
    Carve c(ws);
    const size_t kb = wide_keys(g->depth) ? 8 : 4;
    *ctl = c.take<Control>(1);
    sort_carve(c, *w, n, 64, cfg);  // sized for the widest key
    *a = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    *b = c.take<char>((size_t)(n > 0 ? n : 1) * kb);
    return c.size();
}

size_t cga_sort_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    return max_over_cfgs([&](const SortCfg &c) {
        Control *ctl;
        SortWs w;
        void *a, *b;
        return sort_api_layout(nullptr, g, n, c, &ctl, &w, &a, &b);
    });
}

int cga_sort_keys(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint32_t key_bits, void *d_out, void *d_ws, size_t ws_bytes,
                  const cga_tune *tune, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || !d_ws) return CGA_EINVAL;
    const bool wide = wide_keys(g->depth);
    if (key_bits == 0) key_bits = 3 * g->depth;
    if (key_bits > (wide ? 64u : 32u)) return CGA_EINVAL;
    if (n > 0 && (!d_keys || !d_out)) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    SortCfg cfg;
    CGA_TRY(pick_cfg(tune, wide, n, &cfg, (int)key_bits));
    Control *ctl;
    SortWs w;
    void *a, *b;
    size_t need = sort_api_layout(d_ws, g, n, cfg, &ctl, &w, &a, &b);
    if (ws_bytes < need) return CGA_EWORKSPACE;
    w.passes = sort_passes((int)key_bits, cfg.radix_bits);
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(ctl, w.hist, sort_zero_bytes(w), nullptr, 0, nullptr, s));
    if (n > 0) {
        const void *src = d_keys;
        if (w.passes == 1 && d_keys == d_out) {  // one pass cannot run in place
            CGA_HIP(hipMemcpyAsync(a, d_keys, (size_t)n * (wide ? 8 : 4),
                                   hipMemcpyDeviceToDevice, s));
            src = a;
        }
        if (w.passes == 0) {
            if (d_out != d_keys)
                CGA_HIP(hipMemcpyAsync(d_out, d_keys, (size_t)n * (wide ? 8 : 4),
                                       hipMemcpyDeviceToDevice, s));
        } else if (wide) {
            sort_launch<uint64_t>(w, (const uint64_t *)src, (uint64_t *)d_out, (uint64_t *)a,
                                  (uint64_t *)b, n, d_n, false, ctl->tile_ctr, s);
        } else {
            sort_launch<uint32_t>(w, (const uint32_t *)src, (uint32_t *)d_out, (uint32_t *)a,
                                  (uint32_t *)b, n, d_n, false, ctl->tile_ctr, s);
        }
        CGA_HIP(hipGetLastError());
    }
    return CGA_OK;
}

// ------------------------------------------------------------ paper arrays
size_t cga_to_arrays_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    return arrays_layout(nullptr, g, n).bytes;
}

int cga_to_arrays(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n,
                  uint32_t *d_x_index, int64_t *d_x_ptr, uint32_t *d_y_index, int64_t *d_y_ptr,
                  uint32_t *d_z_index, int64_t *d_n_x, int64_t *d_n_xy, int64_t *n_x_host,
                  int64_t *n_xy_host, void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || !d_ws) return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_LINEAR) return CGA_EMISMATCH;
    if (!d_x_ptr || !d_y_ptr) return CGA_EINVAL;
    if (n > 0 && (!d_keys || !d_x_index || !d_y_index || !d_z_index)) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    ArraysLayout L = arrays_layout(d_ws, g, n);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int64_t *nx = d_n_x ? d_n_x : &L.ctl->count;
    int64_t *nxy = d_n_xy ? d_n_xy : &L.ctl->count2;
    // the pointer arrays start at 0 even when there are no voxels
    CGA_TRY(launch_begin(L.ctl, L.st_xy, (size_t)rle_tiles(n) * 8, L.st_x,
                         (size_t)rle_tiles(n) * 8, nx, s, nxy, d_x_ptr, d_y_ptr));
    if (n > 0) {
        if (wide_keys(g->depth))
            arrays_enqueue<uint64_t>(g, (const uint64_t *)d_keys, n, d_n, d_x_index, d_x_ptr,
                                     d_y_index, d_y_ptr, d_z_index, nx, nxy, L, s);
        else
            arrays_enqueue<uint32_t>(g, (const uint32_t *)d_keys, n, d_n, d_x_index, d_x_ptr,
                                     d_y_index, d_y_ptr, d_z_index, nx, nxy, L, s);
        CGA_HIP(hipGetLastError());
    }
    if (n_x_host || n_xy_host) {
        int st = finish_sync(L.ctl, s);
        if (n_x_host) CGA_TRY(read_count(nx, n_x_host, s));
        if (n_xy_host) CGA_TRY(read_count(nxy, n_xy_host, s));
        return st;
    }
    return CGA_OK;
}

}  // extern "C"
