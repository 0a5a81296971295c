// Attribute payload: the Value array of Section V.
//
// Per-voxel values from per-point ones, with no atomics: the points' keys
// (quantize + encode) and their packed attributes are radix-sorted together
// (a key-value onesweep), so each voxel's points become one run of equal
// keys; one pass then numbers the runs (heads counted with a decoupled
// look-back), sums each run's four channels and its length, and writes the
// run's value -- the channel averages rounded half up, floor((2 sum + count)
// / (2 count)), the colour averaging of the grid downsampling in Section
// III-B -- at the run's rank, checking that the run's key is the CGA key
// there.  A run that crosses tile boundaries leaves one record per tile it
// touches; the tile holding its head adds them up in a second, small pass.
//
// Values of a merge, Eq. (1): every key of the union looks itself up in both
// inputs; a key in both takes the base cloud's value or the channel average
// of the two (the two choices of Section II-A).
#include "cga_common.h"
#include "cga_encode.h"
#include "cga_sort.h"

namespace cga {

template <typename K>
__device__ __forceinline__ int64_t lower_bound_keys(const K *keys, int64_t n, uint64_t q) {
    int64_t lo = 0, len = n;
    while (len > 0) {
        const int64_t half = len >> 1;
        if ((uint64_t)keys[lo + half] < q) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

__device__ __forceinline__ uint32_t round_half_up(uint64_t sum, uint64_t count) {
    return (uint32_t)((2 * sum + count) / (2 * count));
}

constexpr int kValBlock = 256;
constexpr int kValItems = 16;
constexpr int kValTile = kValBlock * kValItems;
constexpr uint32_t kRecFirstCont = 1u;   // the tile's first run began in an earlier tile
constexpr uint32_t kRecFirstEnds = 2u;   // ... and ends inside this tile
constexpr uint32_t kRecLastOwns = 4u;    // the tile's last run began here and continues past it

inline int64_t val_tiles(int64_t n) { return n <= 0 ? 1 : (n + kValTile - 1) / kValTile; }

// Four channel sums, then the point count.
struct VSum {
    uint64_t c[5];
};

__device__ __forceinline__ void vsum_zero(VSum &a) {
#pragma unroll
    for (int q = 0; q < 5; ++q) a.c[q] = 0;
}
__device__ __forceinline__ void vsum_add_attr(VSum &a, uint32_t v) {
#pragma unroll
    for (int q = 0; q < 4; ++q) a.c[q] += (v >> (8 * q)) & 0xFFu;
    a.c[4] += 1;
}
__device__ __forceinline__ void vsum_add(VSum &a, const VSum &b) {
#pragma unroll
    for (int q = 0; q < 5; ++q) a.c[q] += b.c[q];
}

// Per-tile record of the runs that cross its edges.
struct ValRec {
    int64_t first_r, last_r;  // run numbers of the tile's first and last items
    VSum first_sum;           // the first run's sums over this tile (kRecFirstCont)
    VSum last_sum;            // the last run's sums over this tile (kRecLastOwns)
    uint32_t flags, pad;
};

template <typename K>
__device__ __forceinline__ void value_out(int64_t r, uint64_t key, const VSum &a, const K *ukeys,
                                          int64_t u, uint32_t *values, uint32_t *err) {
    if (r < 0 || r >= u || (uint64_t)ukeys[r] != key) {  // a point's voxel is not the CGA key here
        set_err(err, ERR_MISMATCH);
        return;
    }
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v |= round_half_up(a.c[q], a.c[4]) << (8 * q);
    values[r] = v;
}

// Segmented inclusive scan over the threads of the block: element (f, v),
// (f1, v1) + (f2, v2) = (f1 | f2, f2 ? v2 : v1 + v2).  Returns the exclusive
// prefix of this thread (f, v) and the block total.
__device__ __forceinline__ void seg_scan_block(bool f, const VSum &v, bool *ex_f, VSum *ex_v,
                                               bool *tot_f, VSum *tot_v, bool *s_f, VSum *s_v) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    bool inf = f;
    VSum inv = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const bool pf = __shfl_up((int)inf, o, 64) != 0;
        VSum pv;
#pragma unroll
        for (int q = 0; q < 5; ++q) pv.c[q] = __shfl_up(inv.c[q], o, 64);
        if (lane >= o) {
            if (!inf) vsum_add(inv, pv);
            inf = inf || pf;
        }
    }
    if (lane == 63) {
        s_f[wave] = inf;
        s_v[wave] = inv;
    }
    __syncthreads();
    // the waves before this one, combined in order
    bool wf = false;
    VSum wv;
    vsum_zero(wv);
    for (int w = 0; w < wave; ++w) {
        if (s_f[w]) wv = s_v[w];
        else vsum_add(wv, s_v[w]);
        wf = wf || s_f[w];
    }
    // exclusive within the wave: the inclusive value of the lane before
    bool lf = __shfl_up((int)inf, 1, 64) != 0;
    VSum lv;
#pragma unroll
    for (int q = 0; q < 5; ++q) lv.c[q] = __shfl_up(inv.c[q], 1, 64);
    if (lane == 0) {
        lf = false;
        vsum_zero(lv);
    }
    // this thread's exclusive prefix = (waves before) + (lanes before)
    *ex_f = wf || lf;
    if (lf) *ex_v = lv;
    else {
        *ex_v = wv;
        vsum_add(*ex_v, lv);
    }
    bool tf = false;
    VSum tv;
    vsum_zero(tv);
    for (int w = 0; w < kValBlock / 64; ++w) {
        if (s_f[w]) tv = s_v[w];
        else vsum_add(tv, s_v[w]);
        tf = tf || s_f[w];
    }
    *tot_f = tf;
    *tot_v = tv;
    __syncthreads();
}

// One tile of the sorted (key, attribute) pairs: number the runs, finish
// every run whose head and tail both lie in the tile, record the sums of the
// runs that cross its edges.
template <typename K>
__global__ __launch_bounds__(kValBlock) void k_values_runs(
    const K *__restrict__ sk, const uint32_t *__restrict__ sa, int64_t n, const K *__restrict__ ukeys,
    int64_t u_host, const int64_t *d_u, uint32_t *__restrict__ values, ValRec *__restrict__ recs,
    uint64_t *status, int64_t *total_runs, uint32_t *tile_ctr, uint32_t *err) {
    __shared__ uint32_t s_tile;
    __shared__ K s_k[kValTile + 2 + (kValTile + 2) / 16 + 1];
#define SK(j) s_k[(j) + ((j) >> 4)]
    __shared__ uint32_t s_a[kValTile + kValTile / 16 + 1];
#define SA(j) s_a[(j) + ((j) >> 4)]
    __shared__ uint32_t s_wc[kValBlock / 64];
    __shared__ bool s_sf[kValBlock / 64];
    __shared__ VSum s_sv[kValBlock / 64];
    __shared__ int64_t s_pre;
    const int tid = threadIdx.x;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const int64_t base = (int64_t)tile * kValTile;
    if (base >= n) return;
    const int64_t u = dev_count(u_host, d_u) < u_host ? dev_count(u_host, d_u) : u_host;
    {
        K kv[kValItems];
        uint32_t av[kValItems];
#pragma unroll
        for (int it = 0; it < kValItems; ++it) {
            const int64_t i = base + it * kValBlock + tid;
            kv[it] = i < n ? sk[i] : K(0);
            av[it] = i < n ? sa[i] : 0u;
        }
#pragma unroll
        for (int it = 0; it < kValItems; ++it) {
            const int j = it * kValBlock + tid;
            SK(1 + j) = kv[it];
            SA(j) = av[it];
        }
    }
    if (tid == 0) SK(0) = base > 0 ? sk[base - 1] : K(0);
    if (tid == 1) SK(kValTile + 1) = base + kValTile < n ? sk[base + kValTile] : K(0);
    __syncthreads();

    // heads and tails of this thread's 16 consecutive items
    const int j0 = tid * kValItems;
    uint32_t hbits = 0, tbits = 0, hc = 0;
#pragma unroll
    for (int it = 0; it < kValItems; ++it) {
        const int j = j0 + it;
        const int64_t i = base + j;
        if (i < n) {
            if (i == 0 || SK(1 + j) != SK(j)) {
                hbits |= 1u << it;
                ++hc;
            }
            if (i == n - 1 || SK(1 + j) != SK(2 + j)) tbits |= 1u << it;
        }
    }
    uint32_t tot_c;
    const uint32_t ex_c = block_excl_sum<kValBlock>(hc, s_wc, &tot_c);
    if (tid < 64) {  // wave 0: run numbers of the earlier tiles
        int64_t pre = 0;
        if (tile == 0) {
            if (tid == 0) st_agent(&status[tile], (uint64_t)((2ull << 62) | tot_c));
        } else {
            if (tid == 0) st_agent(&status[tile], (uint64_t)((1ull << 62) | tot_c));
            pre = (int64_t)lookback_sum62(status, tile, 0);
            if (tid == 0) st_agent(&status[tile], (uint64_t)((2ull << 62) | (uint64_t)(pre + tot_c)));
        }
        if (tid == 0) {
            s_pre = pre;
            if (base + kValTile >= n && total_runs) *total_runs = pre + tot_c;
        }
    }
    __syncthreads();
    const int64_t pre = s_pre;

    // walk this thread's items: finish runs that start and end here, keep
    // the sums of the leading segment (before the first head) and of the
    // trailing one (from the last head on)
    int64_t r = pre + ex_c - 1;  // run number of the item just before this thread's first head
    VSum cur, lead;
    vsum_zero(cur);
    vsum_zero(lead);
    bool started = false, lead_ends = false, any = false;
    int64_t lead_r = r;
    uint64_t lead_key = 0;
#pragma unroll
    for (int it = 0; it < kValItems; ++it) {
        const int j = j0 + it;
        if (base + j >= n) break;
        any = true;
        if ((hbits >> it) & 1u) {
            ++r;
            started = true;
            vsum_zero(cur);
        }
        vsum_add_attr(cur, SA(j));
        if ((tbits >> it) & 1u) {
            if (started) {
                value_out(r, (uint64_t)SK(1 + j), cur, ukeys, u, values, err);
            } else {
                lead = cur;
                lead_ends = true;
                lead_r = r;
                lead_key = (uint64_t)SK(1 + j);
            }
            vsum_zero(cur);
            started = false;  // items after a tail begin with a head
        }
    }
    // leading segment that does not end in this thread: all of the thread
    if (any && !lead_ends && hbits == 0) lead = cur;
    // scan element: (thread has a head, sums of its open trailing segment, or
    // of all its items when it has no head)
    const bool f = hbits != 0;
    VSum trail = cur;  // the open segment at the end (zero when the last item was a tail)
    bool ex_f, tot_f;
    VSum ex_v, tot_v;
    seg_scan_block(f, trail, &ex_f, &ex_v, &tot_f, &tot_v, s_sf, s_sv);
    if (lead_ends) {
        VSum a = ex_v;
        vsum_add(a, lead);
        if (ex_f) {
            value_out(lead_r, lead_key, a, ukeys, u, values, err);
        } else {  // the tile's first run, begun in an earlier tile
            ValRec &rec = recs[tile];
            rec.first_sum = a;
        }
    }
    if (tid == 0) {
        // the record's bookkeeping: first / last run numbers and flags
        const int64_t tile_end = base + kValTile < n ? base + kValTile : n;
        const bool first_head = base == 0 || SK(1) != SK(0);
        const int jl = (int)(tile_end - 1 - base);
        const bool last_tail = tile_end == n || SK(1 + jl) != SK(2 + jl);
        ValRec &rec = recs[tile];
        rec.first_r = first_head ? pre : pre - 1;
        rec.last_r = pre + tot_c - 1;
        uint32_t fl = 0;
        if (!first_head) {
            fl |= kRecFirstCont;
            if (tot_c == 0 && !last_tail) rec.first_sum = tot_v;  // the whole tile, and the run goes on
            else fl |= kRecFirstEnds;  // its sums came from the thread holding its tail
        }
        if (!last_tail && tot_c > 0) {
            fl |= kRecLastOwns;
            rec.last_sum = tot_v;
        }
        rec.flags = fl;
    }
#undef SK
#undef SA
}

// Runs that cross tile edges: the tile holding the head adds the sums the
// following tiles recorded until the run ends.
template <typename K>
__global__ __launch_bounds__(256) void k_values_cross(const K *__restrict__ sk, int64_t n,
                                                      const K *__restrict__ ukeys, int64_t u_host,
                                                      const int64_t *d_u, const ValRec *__restrict__ recs,
                                                      int64_t tiles, uint32_t *__restrict__ values,
                                                      uint32_t *err) {
    const int64_t u = dev_count(u_host, d_u) < u_host ? dev_count(u_host, d_u) : u_host;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        if ((int64_t)t * kValTile >= n) continue;
        const ValRec &rec = recs[t];
        if (!(rec.flags & kRecLastOwns)) continue;
        VSum a = rec.last_sum;
        int64_t t2 = t + 1;
        for (; t2 < tiles && t2 * kValTile < n; ++t2) {
            const ValRec &nx = recs[t2];
            vsum_add(a, nx.first_sum);
            if (nx.flags & kRecFirstEnds) break;
        }
        const int64_t end = (t + 1) * kValTile;  // first item after tile t: in the run
        value_out(rec.last_r, (uint64_t)sk[end - 1], a, ukeys, u, values, err);
    }
}

// Every CGA key must have a run: the run count equals u.
__global__ void k_values_check(const int64_t *total_runs, int64_t u_host, const int64_t *d_u,
                               uint32_t *err) {
    const int64_t u = dev_count(u_host, d_u) < u_host ? dev_count(u_host, d_u) : u_host;
    if (threadIdx.x == 0 && blockIdx.x == 0 && *total_runs != u) set_err(err, ERR_MISMATCH);
}

template <typename K>
__global__ __launch_bounds__(256) void k_merge_values(
    const K *__restrict__ ka, const uint32_t *__restrict__ va, int64_t na_host, const int64_t *d_na,
    const K *__restrict__ kb, const uint32_t *__restrict__ vb, int64_t nb_host, const int64_t *d_nb,
    const K *__restrict__ km, int64_t nm_host, const int64_t *d_nm, int policy,
    uint32_t *__restrict__ vm, uint32_t *err) {
    auto count = [](int64_t h, const int64_t *d) {
        const int64_t c = dev_count(h, d);
        return c < h ? c : h;
    };
    const int64_t na = count(na_host, d_na), nb = count(nb_host, d_nb), nm = count(nm_host, d_nm);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nm;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = km[j];
        const int64_t ia = lower_bound_keys(ka, na, key), ib = lower_bound_keys(kb, nb, key);
        const bool in_a = ia < na && (uint64_t)ka[ia] == key, in_b = ib < nb && (uint64_t)kb[ib] == key;
        uint32_t v = 0;
        if (in_a && in_b) {
            const uint32_t x = va[ia], y = vb[ib];
            if (policy == CGA_VALUES_AVERAGE) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    v |= round_half_up(((x >> (8 * c)) & 0xFFu) + ((y >> (8 * c)) & 0xFFu), 2) << (8 * c);
            } else {
                v = x;
            }
        } else if (in_a) {
            v = va[ia];
        } else if (in_b) {
            v = vb[ib];
        } else {
            set_err(err, ERR_MISMATCH);
        }
        vm[j] = v;
    }
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

struct ValuesLayout {
    Control *ctl;
    SortWs sort;
    void *ka, *kb;
    uint32_t *va, *vb;
    ValRec *recs;
    uint64_t *status;
    size_t bytes;
};

static ValuesLayout values_layout(void *ws, const cga_grid *g, int64_t n) {
    ValuesLayout L;
    Carve c(ws);
    const size_t kbytes = wide_keys(g->depth) ? 8 : 4, m = (size_t)(n > 0 ? n : 1);
    SortCfg cfg;
    cfg.radix_bits = 8;
    cfg.items = 16;
    L.ctl = c.take<Control>(1);
    sort_carve(c, L.sort, n, 3 * (int)g->depth, cfg);
    L.ka = c.take<char>(m * kbytes);
    L.kb = c.take<char>(m * kbytes);
    L.va = c.take<uint32_t>(m);
    L.vb = c.take<uint32_t>(m);
    L.recs = c.take<ValRec>((size_t)val_tiles(n));
    L.status = c.take<uint64_t>((size_t)val_tiles(n));
    L.bytes = c.size();
    return L;
}

template <typename K>
static void values_enqueue(const cga_grid *g, const float *xyz, int64_t n, const uint32_t *attr,
                           const K *ukeys, int64_t u, const int64_t *d_u, uint32_t *values,
                           const ValuesLayout &L, hipStream_t s) {
    const SortWs &w = L.sort;
    K *a = (K *)L.ka, *b = (K *)L.kb;
    encode_dispatch<K>(g, xyz, n, a, 8, w.passes, w.hist, &L.ctl->err, s);
    // key chain a -> ... -> fin, payload chain attr -> ... -> vfin (as sort_chain)
    K *fin = (w.passes & 1) ? b : a, *other = (w.passes & 1) ? a : b;
    uint32_t *vfin = (w.passes & 1) ? L.vb : L.va, *vother = (w.passes & 1) ? L.va : L.vb;
    const uint32_t *vsorted = attr;
    if (w.passes > 0) {
        sort_launch_kv<K>(w, a, fin, other, fin, attr, vfin, vother, vfin, n, nullptr, true,
                          L.ctl->tile_ctr, s);
        vsorted = vfin;
    } else {
        fin = a;
    }
    const int64_t tiles = val_tiles(n);
    {
        CGA_PROF("values_runs", s);
        k_values_runs<K><<<(unsigned)tiles, kValBlock, 0, s>>>(
            fin, vsorted, n, ukeys, u, d_u, values, L.recs, L.status, &L.ctl->count,
            &L.ctl->tile_ctr[kMaxPasses], &L.ctl->err);
    }
    int64_t blocks = (tiles + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    k_values_cross<K><<<(unsigned)blocks, 256, 0, s>>>(fin, n, ukeys, u, d_u, L.recs, tiles, values,
                                                       &L.ctl->err);
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_voxel_values_workspace_bytes(const cga_grid *g, int64_t n) {
    if (!grid_valid(g) || n < 0) return 0;
    return values_layout(nullptr, g, n).bytes;
}

int cga_voxel_values(const cga_grid *g, const float *d_xyz, int64_t n, const uint32_t *d_attr,
                     const void *d_keys, int64_t u, const int64_t *d_u, uint32_t *d_values,
                     void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || u < 0 || !d_ws) return CGA_EINVAL;
    if ((n > 0 && (!d_xyz || !d_attr)) || (u > 0 && (!d_keys || !d_values))) return CGA_EINVAL;
    if (n >= (int64_t)1 << 30) return CGA_EUNSUPPORTED;
    ValuesLayout L = values_layout(d_ws, g, n);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(L.ctl, L.sort.hist, sort_zero_bytes(L.sort), L.status,
                         (size_t)val_tiles(n) * 8, nullptr, s));
    if (n > 0) {
        if (wide_keys(g->depth))
            values_enqueue<uint64_t>(g, d_xyz, n, d_attr, (const uint64_t *)d_keys, u, d_u, d_values,
                                     L, s);
        else
            values_enqueue<uint32_t>(g, d_xyz, n, d_attr, (const uint32_t *)d_keys, u, d_u, d_values,
                                     L, s);
    }
    // every key must have had a run of points (the run count is u)
    k_values_check<<<1, 64, 0, s>>>(&L.ctl->count, u, d_u, &L.ctl->err);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

size_t cga_merge_values_workspace_bytes(void) { return sizeof(Control) < 256 ? 256 : sizeof(Control); }

int cga_merge_values(const cga_grid *g, const void *d_keys_a, const uint32_t *d_values_a, int64_t na,
                     const int64_t *d_na, const void *d_keys_b, const uint32_t *d_values_b,
                     int64_t nb, const int64_t *d_nb, const void *d_keys_m, int64_t nm,
                     const int64_t *d_nm, int policy, uint32_t *d_values_m, void *d_ws,
                     size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || na < 0 || nb < 0 || nm < 0 || !d_ws) return CGA_EINVAL;
    if (policy != CGA_VALUES_BASE && policy != CGA_VALUES_AVERAGE) return CGA_EINVAL;
    if ((na > 0 && (!d_keys_a || !d_values_a)) || (nb > 0 && (!d_keys_b || !d_values_b)) ||
        (nm > 0 && (!d_keys_m || !d_values_m)))
        return CGA_EINVAL;
    if (ws_bytes < cga_merge_values_workspace_bytes()) return CGA_EWORKSPACE;
    Control *ctl = (Control *)d_ws;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (nm > 0) {
        CGA_PROF("merge_values", s);
        if (wide_keys(g->depth))
            k_merge_values<uint64_t><<<grid_for(nm), 256, 0, s>>>(
                (const uint64_t *)d_keys_a, d_values_a, na, d_na, (const uint64_t *)d_keys_b,
                d_values_b, nb, d_nb, (const uint64_t *)d_keys_m, nm, d_nm, policy, d_values_m,
                &ctl->err);
        else
            k_merge_values<uint32_t><<<grid_for(nm), 256, 0, s>>>(
                (const uint32_t *)d_keys_a, d_values_a, na, d_na, (const uint32_t *)d_keys_b,
                d_values_b, nb, d_nb, (const uint32_t *)d_keys_m, nm, d_nm, policy, d_values_m,
                &ctl->err);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
