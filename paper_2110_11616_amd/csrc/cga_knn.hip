// k-nearest-neighbour search, Eq. (7)-(8) generalised to k, over a sorted
// unique MORTON key array, and plain binary-search point lookup.
//
// Morton keys make every octree cell a contiguous key range: cell (prefix,
// L) holds exactly the keys in [prefix << 3L, (prefix + 1) << 3L).  A query
// (one thread each) first takes the keys around its own key's insertion point
// as candidates, which bounds the k-th squared distance by some D.  Every
// better point then lies in the box of half-width floor(sqrt(D)) around the
// query, which at most 2 x 2 x 2 cells of the smallest level whose cell edge
// covers the box contain.  Each such cell is walked in key order as an
// implicit octree without a stack: a cell whose nearest point is farther
// than the current k-th distance is skipped (strictly farther, so ties
// survive), a cell with at most kScan keys is scanned exactly, any other is
// split into its eight children.  The key array position of the next cell
// is found by galloping search from the current one.  Candidates are kept in
// registers ordered by (squared distance, key); key order is array order.
#include "cga_common.h"

namespace cga {

constexpr int kKnnBlock = 256;
constexpr int kScan = 16;  // scan a cell outright when it holds at most this many keys

struct Cand {
    uint64_t d;
    int32_t i;
};

__device__ __forceinline__ bool cand_lt(uint64_t d, int32_t i, const Cand &c) {
    return d < c.d || (d == c.d && i < c.i);
}

// Ascending list of KT candidates, the last KT - k of which are the answer;
// the first slots hold (0, -1) sentinels that no real candidate precedes.
template <int KT>
__device__ __forceinline__ void cand_insert(Cand (&e)[KT], uint64_t d, int32_t i) {
    if (!cand_lt(d, i, e[KT - 1])) return;
    bool placed = false;
#pragma unroll
    for (int s = KT - 1; s > 0; --s) {
        const bool sh = !placed && cand_lt(d, i, e[s - 1]);
        Cand nv = sh ? e[s - 1] : (placed ? e[s] : Cand{d, i});
        placed = placed || !sh;
        e[s] = nv;
    }
    if (!placed) e[0] = Cand{d, i};
}

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

// First index >= lo whose key is >= t, given keys[lo - 1] < t.
template <typename K>
__device__ __forceinline__ int64_t gallop(const K *keys, int64_t n, int64_t lo, K t) {
    if (lo >= n || keys[lo] >= t) return lo;
    int64_t prev = lo, step = 1, hi;
    for (;;) {
        int64_t nx = prev + step;
        if (nx >= n) {
            hi = n;
            break;
        }
        if (keys[nx] >= t) {
            hi = nx;
            break;
        }
        prev = nx;
        step <<= 1;
    }
    int64_t a = prev + 1, b = hi;  // answer in [a, b]
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (keys[mid] < t) a = mid + 1;
        else b = mid;
    }
    return a;
}

__device__ __forceinline__ uint64_t sq_dist(const Vox &a, uint32_t x, uint32_t y, uint32_t z) {
    int64_t dx = (int64_t)a.x - x, dy = (int64_t)a.y - y, dz = (int64_t)a.z - z;
    return (uint64_t)(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ uint64_t axis_gap(uint32_t q, uint32_t lo, uint32_t hi) {
    return q < lo ? (uint64_t)(lo - q) : (q > hi ? (uint64_t)(q - hi) : 0ull);
}

__device__ __forceinline__ uint32_t isqrt64(uint64_t v) {
    uint64_t r = (uint64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (uint32_t)r;
}

template <typename K, int KT>
__global__ __launch_bounds__(kKnnBlock) void k_knn(const K *__restrict__ keys, int64_t n_host,
                                                   const int64_t *d_n, const float *__restrict__ q,
                                                   int64_t nq, float o0, float o1, float o2,
                                                   float scale, uint32_t depth, int k,
                                                   int64_t *__restrict__ idx_out,
                                                   uint64_t *__restrict__ d2_out, uint32_t *err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nq) return;
    const int64_t n = dev_count(n_host, d_n);
    const float o[3] = {o0, o1, o2};
    Vox qv;
    if (!quantize3(q[3 * j], q[3 * j + 1], q[3 * j + 2], o, scale, depth, qv)) {
        set_err(err, ERR_NONFINITE);
        for (int s = 0; s < k; ++s) {
            idx_out[j * k + s] = -1;
            d2_out[j * k + s] = ~0ull;
        }
        return;
    }

    Cand e[KT];
#pragma unroll
    for (int s = 0; s < KT; ++s) e[s] = s < KT - k ? Cand{0, -1} : Cand{~0ull, 0x7FFFFFFF};

    // seed: keys around the query's own insertion point
    const K qkey = (K)enc3(qv.x, qv.y, qv.z, depth, false);
    const int64_t p = lower_bound_dev(keys, n, qkey);
    const int64_t w = k > 4 ? k : 4;
    const int64_t seed_lo = p > w ? p - w : 0, seed_hi = p + w < n ? p + w : n;
    for (int64_t i = seed_lo; i < seed_hi; ++i) {
        Vox v = dec3(keys[i], depth, false);
        cand_insert<KT>(e, sq_dist(v, qv.x, qv.y, qv.z), (int32_t)i);
    }

    // start level: cells at least as wide as the box that can still hold a
    // better point
    const uint32_t top = (1u << depth) - 1;
    int ls = (int)depth;
    uint32_t r = 0;
    if (e[KT - 1].d != ~0ull) {
        r = isqrt64(e[KT - 1].d);
        if (r < top) {
            ls = 0;
            while (ls < (int)depth && ((1u << ls) < 2 * r + 1)) ++ls;
        }
    }
    uint32_t clo[3], chi[3];
    {
        const uint32_t qc[3] = {qv.x, qv.y, qv.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint32_t lo = qc[a] > r ? qc[a] - r : 0;
            uint32_t hi = (uint64_t)qc[a] + r < top ? qc[a] + r : top;
            clo[a] = lo >> ls;
            chi[a] = hi >> ls;
        }
    }

    for (uint32_t cx = clo[0]; cx <= chi[0]; ++cx)
        for (uint32_t cy = clo[1]; cy <= chi[1]; ++cy)
            for (uint32_t cz = clo[2]; cz <= chi[2]; ++cz) {
                // walk the subtree of cell (cx, cy, cz) at level ls in key order
                uint64_t prefix = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
                int L = ls;
                int64_t cur = -1;  // lower bound position of the current cell, once known
                for (;;) {
                    bool visit = true;
                    {
                        const uint32_t bx = compact3(prefix >> 2) << L, by = compact3(prefix >> 1) << L,
                                       bz = compact3(prefix) << L;
                        const uint32_t ext = (1u << L) - 1;
                        const uint64_t gx = axis_gap(qv.x, bx, bx + ext), gy = axis_gap(qv.y, by, by + ext),
                                       gz = axis_gap(qv.z, bz, bz + ext);
                        if (gx * gx + gy * gy + gz * gz > e[KT - 1].d) visit = false;
                    }
                    if (visit) {
                        const int sh = 3 * L;
                        const K ks = (K)(prefix << sh);
                        // exclusive end; at most 2^63 since 3 * depth <= 63
                        const uint64_t ke64 = (prefix + 1) << sh;
                        cur = cur < 0 ? lower_bound_dev(keys, n, ks) : gallop(keys, n, cur, ks);
                        auto in_cell = [&](int64_t i) {
                            return i < n && (uint64_t)keys[i] < ke64;
                        };
                        if (in_cell(cur)) {
                            if (L > 0 && in_cell(cur + kScan)) {
                                prefix <<= 3;
                                --L;
                                continue;
                            }
                            for (; in_cell(cur); ++cur) {
                                if (cur >= seed_lo && cur < seed_hi) continue;
                                Vox v = dec3(keys[cur], depth, false);
                                cand_insert<KT>(e, sq_dist(v, qv.x, qv.y, qv.z), (int32_t)cur);
                            }
                        }
                    }
                    while (L < ls && (prefix & 7) == 7) {
                        prefix >>= 3;
                        ++L;
                    }
                    if (L == ls) break;
                    ++prefix;
                }
            }

#pragma unroll
    for (int s = 0; s < KT; ++s) {
        if (s >= KT - k) {
            const int o_ = s - (KT - k);
            const bool real = e[s].d != ~0ull;
            idx_out[j * k + o_] = real ? (int64_t)e[s].i : -1;
            d2_out[j * k + o_] = real ? e[s].d : ~0ull;
        }
    }
}

template <typename K, int KT>
static void knn_launch(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                       const float *q, int64_t nq, int k, int64_t *idx, uint64_t *d2, uint32_t *err,
                       hipStream_t s) {
    k_knn<K, KT><<<(unsigned)((nq + kKnnBlock - 1) / kKnnBlock), kKnnBlock, 0, s>>>(
        keys, n, d_n, q, nq, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth, k, idx,
        d2, err);
}

template <typename K>
static void knn_dispatch(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                         const float *q, int64_t nq, int k, int64_t *idx, uint64_t *d2,
                         uint32_t *err, hipStream_t s) {
    if (k <= 1) knn_launch<K, 1>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
    else if (k <= 2) knn_launch<K, 2>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
    else if (k <= 4) knn_launch<K, 4>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
    else if (k <= 8) knn_launch<K, 8>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
    else if (k <= 16) knn_launch<K, 16>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
    else knn_launch<K, 32>(g, keys, n, d_n, q, nq, k, idx, d2, err, s);
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

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_knn_workspace_bytes(const cga_grid *g, int64_t n, int64_t nq) {
    if (!grid_valid(g) || n < 0 || nq < 0) return 0;
    return kControlBytes;
}

int cga_knn(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n, const float *d_q,
            int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2, void *d_ws, size_t ws_bytes,
            cga_stream stream) {
    if (!grid_valid(g) || n < 0 || nq < 0 || k < 1 || k > 32 || !d_ws) return CGA_EINVAL;
    if (nq > 0 && (!d_q || !d_idx || !d_d2)) return CGA_EINVAL;
    if (n > 0 && !d_keys) return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_MORTON) return CGA_EUNSUPPORTED;
    if (n >= ((int64_t)1 << 31) - 1) return CGA_EUNSUPPORTED;
    if (ws_bytes < kControlBytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Control *ctl = (Control *)d_ws;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (nq > 0) {
        if (wide_keys(g->depth))
            knn_dispatch<uint64_t>(g, (const uint64_t *)d_keys, n, d_n, d_q, nq, k, d_idx, d_d2,
                                   &ctl->err, s);
        else
            knn_dispatch<uint32_t>(g, (const uint32_t *)d_keys, n, d_n, d_q, nq, k, d_idx, d_d2,
                                   &ctl->err, s);
        CGA_HIP(hipGetLastError());
    }
    return CGA_OK;
}

int cga_binary_lookup(const uint64_t *d_keys, int64_t n, const int64_t *d_n, const uint64_t *d_q,
                      int64_t nq, int64_t *d_rank, uint8_t *d_found, cga_stream stream) {
    if (n < 0 || nq < 0) return CGA_EINVAL;
    if ((n > 0 && !d_keys) || (nq > 0 && (!d_q || !d_rank))) return CGA_EINVAL;
    if (nq == 0) return CGA_OK;
    hipStream_t s = (hipStream_t)stream;
    k_binary_lookup<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(d_keys, n, d_n, d_q, nq, d_rank,
                                                                d_found);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
