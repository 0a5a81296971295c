// Temporal prediction of a frame from a reference frame, the inter-frame
// path of the CGA compression scheme (Section V-D), on two CGAs (sorted
// unique keys plus one packed 4 x 8-bit value per voxel):
//
// 1. clustering: k-means over each frame's voxels with eight centres started
//    at the corners of the frame's bounding box (corner i takes the maximum
//    of x when bit 2 of i is set, of y for bit 1, of z for bit 0, else the
//    minimum).  A pass assigns every voxel to its nearest centre (squared
//    distance in double precision, x + y + z terms summed in that order,
//    every operation separately rounded; ties to the lower cluster) while
//    summing coordinates per cluster in 64-bit integers; the run stops at
//    the first pass that changes no assignment or after max_iter passes, and
//    otherwise every non-empty cluster moves to its mean (one rounded
//    division), an empty one stays;
// 2. motion: cluster i of the two frames correspond (same starting corner);
//    its motion vector is the predicted centroid minus the reference one,
//    rounded half away from zero to whole voxels;
// 3. matching: every predicted voxel moved back by its cluster's vector is
//    matched to the reference voxel of least SAD over the four channels among
//    those within `window` voxels on each axis (ties: smaller L1 offset, then
//    smaller key), found by key searches -- one lower bound and a short scan
//    per (x, y) column for LINEAR keys, one search per voxel for MORTON;
// 4. residual: predicted minus matched channels (int16), or the voxel's own
//    channels with match -1 and SAD UINT32_MAX when it left the grid or found
//    no reference voxel.
//
// The passes run as a fixed sequence of launches that turn into no-ops once
// a frame has converged, so the whole call is asynchronous.
#include "cga_common.h"

namespace cga {

constexpr int kCl = 8;  // clusters (the bounding-box corners)
constexpr int kTemporalMaxWindow = 15;
constexpr int kTemporalMaxIter = 1000;

// Per-frame k-means state, zeroed at the start of a call.  Pass t assigns
// with the centres cent[t & 1] and sums into sum / cnt / changed [t % 3]; it
// computes its centres itself, in every block, from pass t - 1's sums (so
// no launch sits between passes), and clears slot (t + 1) % 3, which pass
// t - 1 finished reading.
// Each pass's sums are kept in kRep copies (block b adds to copy b % kRep),
// so that fewer blocks add to one word; the next pass adds the copies up.
// The sums are integers, so the copies change no result.
constexpr int kRep = 8;

struct KmState {
    double cent[2][kCl][3];
    unsigned long long sum[3][kRep][kCl][3];
    unsigned long long cnt[3][kRep][kCl];
    uint32_t changed[3];
    uint32_t lo_inv[3];  // ~min per axis (so that a zeroed block starts at "no voxel")
    uint32_t hi[3];
    uint32_t halt;       // the run has ended: later passes do nothing
    int32_t iters;       // passes run
};

template <typename K>
__device__ __forceinline__ int64_t lower_bound_k(const K *keys, int64_t n, uint64_t v) {
    int64_t lo = 0, len = n;
    while (len > 0) {
        const int64_t half = len >> 1;
        if ((uint64_t)keys[lo + half] < v) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// Frame f (blockIdx.y) of the two: keys, count.
template <typename K>
struct Frames {
    const K *keys[2];
    int64_t n[2];
    uint8_t *assign[2];
};

template <typename K>
__global__ __launch_bounds__(256) void k_km_bbox(Frames<K> F, uint32_t depth, bool linear, KmState *st) {
    const int f = blockIdx.y;
    uint32_t lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.n[f];
         i += (int64_t)gridDim.x * blockDim.x) {
        const Vox v = dec3((uint64_t)F.keys[f][i], depth, linear);
        const uint32_t c[3] = {v.x, v.y, v.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = c[a] < lo[a] ? c[a] : lo[a];
            hi[a] = c[a] > hi[a] ? c[a] : hi[a];
        }
    }
    // wave, then block, then one atomic per block and value
    __shared__ uint32_t s_m[6];
    if (threadIdx.x < 6) s_m[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint32_t l = ~lo[a], h = hi[a];
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t lo2 = __shfl_xor(l, o, 64), h2 = __shfl_xor(h, o, 64);
            l = lo2 > l ? lo2 : l;
            h = h2 > h ? h2 : h;
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMax(&s_m[a], l);
            atomicMax(&s_m[3 + a], h);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMax(&st[f].lo_inv[threadIdx.x], s_m[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&st[f].hi[threadIdx.x - 3], s_m[threadIdx.x]);
}

__global__ void k_km_seed(KmState *st) {
    const int f = blockIdx.x, c = threadIdx.x;
    if (c < kCl) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint32_t lo = ~st[f].lo_inv[a], hi = st[f].hi[a];
            if (lo > hi) lo = hi = 0;  // an empty frame: every corner at the origin
            st[f].cent[0][c][a] = (double)(((c >> (2 - a)) & 1) ? hi : lo);
        }
    }
}

// One pass over both frames: stop if the previous pass changed nothing,
// else move to the previous pass's cluster means and assign every voxel.
template <typename K>
__global__ __launch_bounds__(256) void k_km_assign(Frames<K> F, uint32_t depth, bool linear, int pass,
                                                   KmState *st) {
    const int f = blockIdx.y;
    KmState &S = st[f];
    if (S.halt) return;  // block-uniform
    const int cur = pass % 3, prev = (pass + 2) % 3, next = (pass + 1) % 3;
    if (pass > 0 && !S.changed[prev]) {  // the run ended with the previous pass
        if (blockIdx.x == 0 && threadIdx.x == 0) S.halt = 1;
        return;
    }
    __shared__ unsigned long long s_sum[kCl * 4];
    __shared__ uint32_t s_changed;
    for (int t = threadIdx.x; t < kCl * 4; t += blockDim.x) s_sum[t] = 0;
    if (threadIdx.x == 0) s_changed = 0;
    // pass 0 starts from the corners in cent[0]; pass t > 0 from the means
    // of pass t - 1's clusters, an empty cluster keeping pass t - 1's centre
    // (24 lanes divide, the block reads the results from LDS)
    __shared__ double s_c[kCl * 3];
    if (threadIdx.x < kCl * 3) {
        const int k = threadIdx.x / 3, a = threadIdx.x % 3;
        const int before = pass > 0 ? (pass + 1) & 1 : 0;
        unsigned long long n = 0, sa = 0;
        if (pass > 0)
#pragma unroll
            for (int r = 0; r < kRep; ++r) {
                n += S.cnt[prev][r][k];
                sa += S.sum[prev][r][k][a];
            }
        const double v = n > 0 ? __ddiv_rn((double)sa, (double)n) : S.cent[before][k][a];
        s_c[threadIdx.x] = v;
        // block 0 keeps this pass's centres (for the next pass's empty
        // clusters and for the result)
        if (blockIdx.x == 0 && pass > 0) S.cent[pass & 1][k][a] = v;
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) S.iters = pass + 1;
        for (int t = threadIdx.x; t < kRep * kCl * 4; t += blockDim.x) {
            const int r = t / (kCl * 4), w = t % (kCl * 4);
            if ((w & 3) == 3) S.cnt[next][r][w >> 2] = 0;
            else S.sum[next][r][w >> 2][w & 3] = 0;
        }
        if (threadIdx.x == 0) S.changed[next] = 0;
    }
    __syncthreads();
    double c[kCl][3];
#pragma unroll
    for (int k = 0; k < kCl; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) c[k][a] = s_c[k * 3 + a];
    bool changed = false;
    const int lane = threadIdx.x & 63;
    // whole waves step together, so that the sums can be gathered per wave:
    // neighbouring keys are neighbouring voxels, so a wave rarely spans more
    // than one or two clusters, and each cluster costs one reduction
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < F.n[f]; base += waves * 64) {
        const int64_t i = base + lane;
        const bool active = i < F.n[f];
        Vox v{0, 0, 0};
        int best = 0;
        if (active) {
            v = dec3((uint64_t)F.keys[f][i], depth, linear);
            const double px = (double)v.x, py = (double)v.y, pz = (double)v.z;
            double bd = 0.0;
#pragma unroll
            for (int k = 0; k < kCl; ++k) {
                const double dx = __dsub_rn(px, c[k][0]), dy = __dsub_rn(py, c[k][1]),
                             dz = __dsub_rn(pz, c[k][2]);
                const double d = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                if (k == 0 || d < bd) {
                    bd = d;
                    best = k;
                }
            }
            if (pass == 0 || F.assign[f][i] != best) changed = true;
            F.assign[f][i] = (uint8_t)best;
        }
        uint64_t rem = __ballot(active);
        while (rem) {
            const int leader = __ffsll((unsigned long long)rem) - 1;
            const int k = __shfl(best, leader, 64);
            const bool mine = active && best == k;
            const uint64_t m = __ballot(mine);
            // at most 64 coordinates below 2^21 each: 32-bit sums are exact
            uint32_t sx = mine ? v.x : 0u, sy = mine ? v.y : 0u, sz = mine ? v.z : 0u;
            for (int o = 32; o > 0; o >>= 1) {
                sx += __shfl_xor(sx, o, 64);
                sy += __shfl_xor(sy, o, 64);
                sz += __shfl_xor(sz, o, 64);
            }
            if (lane == leader) {
                atomicAdd(&s_sum[k * 4 + 0], (unsigned long long)sx);
                atomicAdd(&s_sum[k * 4 + 1], (unsigned long long)sy);
                atomicAdd(&s_sum[k * 4 + 2], (unsigned long long)sz);
                atomicAdd(&s_sum[k * 4 + 3], (unsigned long long)__popcll(m));
            }
            rem &= ~m;
        }
    }
    if (__ballot(changed) && (threadIdx.x & 63) == 0) s_changed = 1;
    __syncthreads();
    for (int t = threadIdx.x; t < kCl * 4; t += blockDim.x) {
        const unsigned long long v = s_sum[t];
        const int r = blockIdx.x % kRep;
        if (v) atomicAdd((t & 3) == 3 ? &S.cnt[cur][r][t >> 2] : &S.sum[cur][r][t >> 2][t & 3], v);
    }
    if (threadIdx.x == 0 && s_changed) atomicOr(&S.changed[cur], 1u);
}

// Centroids, motion vectors and pass counts to the caller's arrays.
__global__ void k_motion(const KmState *st, double *centroids, int32_t *mv, int32_t *iters,
                         int32_t *mv_ws) {
    const int t = threadIdx.x;  // cluster * 3 + axis
    if (t < kCl * 3) {
        const int k = t / 3, a = t % 3;
        // the centres of each frame's last pass
        const double cr = st[0].cent[(st[0].iters + 1) & 1][k][a], cp = st[1].cent[(st[1].iters + 1) & 1][k][a];
        const int32_t m = (int32_t)round(__dsub_rn(cp, cr));
        mv_ws[t] = m;
        if (mv) mv[t] = m;
        if (centroids) {
            centroids[t] = cr;
            centroids[kCl * 3 + t] = cp;
        }
    }
    if (t < 2 && iters) iters[t] = st[t].iters;
}

__device__ __forceinline__ uint32_t chan_sad(uint32_t a, uint32_t b) {
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int32_t d = (int32_t)((a >> (8 * c)) & 0xFFu) - (int32_t)((b >> (8 * c)) & 0xFFu);
        s += (uint32_t)(d < 0 ? -d : d);
    }
    return s;
}

template <typename K>
__global__ __launch_bounds__(256) void k_match(const K *__restrict__ ref_keys,
                                               const uint32_t *__restrict__ ref_vals, int64_t n_ref,
                                               const K *__restrict__ pred_keys,
                                               const uint32_t *__restrict__ pred_vals, int64_t n_pred,
                                               const uint8_t *__restrict__ pred_assign,
                                               const int32_t *__restrict__ mv_ws, uint32_t depth,
                                               bool linear, int window, int64_t *__restrict__ match,
                                               uint32_t *__restrict__ sad, int16_t *__restrict__ residual) {
    __shared__ int32_t s_mv[kCl * 3];
    if (threadIdx.x < kCl * 3) s_mv[threadIdx.x] = mv_ws[threadIdx.x];
    __syncthreads();
    const int64_t top = (int64_t)1 << depth;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pred;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Vox p = dec3((uint64_t)pred_keys[i], depth, linear);
        const int cl = pred_assign[i];
        const int64_t r[3] = {(int64_t)p.x - s_mv[cl * 3], (int64_t)p.y - s_mv[cl * 3 + 1],
                              (int64_t)p.z - s_mv[cl * 3 + 2]};
        const uint32_t pv = pred_vals[i];
        int64_t best = -1;
        uint32_t bs = 0xFFFFFFFFu, bl = 0;
        uint64_t bk = 0;
        auto consider = [&](int64_t j, uint32_t l1) __attribute__((always_inline)) {
            const uint32_t s = chan_sad(pv, ref_vals[j]);
            const uint64_t key = (uint64_t)ref_keys[j];
            if (best < 0 || s < bs || (s == bs && (l1 < bl || (l1 == bl && key < bk)))) {
                best = j;
                bs = s;
                bl = l1;
                bk = key;
            }
        };
        const bool inside = r[0] >= 0 && r[0] < top && r[1] >= 0 && r[1] < top && r[2] >= 0 && r[2] < top;
        if (inside && n_ref > 0) {
            const int64_t zlo = r[2] - window > 0 ? r[2] - window : 0;
            const int64_t zhi = r[2] + window < top - 1 ? r[2] + window : top - 1;
            for (int64_t x = r[0] - window; x <= r[0] + window; ++x) {
                if (x < 0 || x >= top) continue;
                for (int64_t y = r[1] - window; y <= r[1] + window; ++y) {
                    if (y < 0 || y >= top) continue;
                    const uint32_t lxy = (uint32_t)((x > r[0] ? x - r[0] : r[0] - x) + (y > r[1] ? y - r[1] : r[1] - y));
                    if (linear) {
                        // the column's z range is one run of LINEAR keys
                        const uint64_t k0 = enc3((uint32_t)x, (uint32_t)y, (uint32_t)zlo, depth, true);
                        const uint64_t k1 = enc3((uint32_t)x, (uint32_t)y, (uint32_t)zhi, depth, true);
                        for (int64_t j = lower_bound_k(ref_keys, n_ref, k0); j < n_ref && (uint64_t)ref_keys[j] <= k1; ++j) {
                            const int64_t z = (int64_t)((uint64_t)ref_keys[j] & (uint64_t)(top - 1));
                            consider(j, lxy + (uint32_t)(z > r[2] ? z - r[2] : r[2] - z));
                        }
                    } else {
                        for (int64_t z = zlo; z <= zhi; ++z) {
                            const uint64_t key = enc3((uint32_t)x, (uint32_t)y, (uint32_t)z, depth, false);
                            const int64_t j = lower_bound_k(ref_keys, n_ref, key);
                            if (j < n_ref && (uint64_t)ref_keys[j] == key)
                                consider(j, lxy + (uint32_t)(z > r[2] ? z - r[2] : r[2] - z));
                        }
                    }
                }
            }
        }
        match[i] = best;
        sad[i] = best < 0 ? 0xFFFFFFFFu : bs;
        const uint32_t rv = best < 0 ? 0u : ref_vals[best];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            residual[4 * i + c] = (int16_t)((int32_t)((pv >> (8 * c)) & 0xFFu) - (int32_t)((rv >> (8 * c)) & 0xFFu));
    }
}

static unsigned temporal_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

struct TemporalLayout {
    Control *ctl;
    KmState *st;
    int32_t *mv;
    size_t bytes;
};

static TemporalLayout temporal_layout(void *ws) {
    TemporalLayout L;
    Carve c(ws);
    L.ctl = c.take<Control>(1);
    L.st = c.take<KmState>(2);
    L.mv = c.take<int32_t>(kCl * 3);
    L.bytes = c.size();
    return L;
}

template <typename K>
static void temporal_launch(const cga_grid *g, const K *rk, const uint32_t *rv, int64_t nr,
                            const K *pk, const uint32_t *pv, int64_t np, int window, int max_iter,
                            uint8_t *ra, uint8_t *pa, double *cent, int32_t *mv, int32_t *iters,
                            int64_t *match, uint32_t *sad, int16_t *res, const TemporalLayout &L,
                            hipStream_t s) {
    const bool linear = g->key_mode == CGA_KEY_LINEAR;
    Frames<K> F{{rk, pk}, {nr, np}, {ra, pa}};
    // a few blocks per CU, striding over the frame: few global atomics per pass
    unsigned gb = temporal_grid(nr > np ? nr : np);
    gb = gb < 512 ? gb : 512;
    const dim3 grid(gb, 2);
    {
        CGA_PROF("temporal_kmeans", s);
        k_km_bbox<K><<<grid, 256, 0, s>>>(F, g->depth, linear, L.st);
        k_km_seed<<<2, 64, 0, s>>>(L.st);
        for (int pass = 0; pass < max_iter; ++pass)
            k_km_assign<K><<<grid, 256, 0, s>>>(F, g->depth, linear, pass, L.st);
        k_motion<<<1, 64, 0, s>>>(L.st, cent, mv, iters, L.mv);
    }
    if (np > 0) {
        CGA_PROF("temporal_match", s);
        k_match<K><<<temporal_grid(np), 256, 0, s>>>(rk, rv, nr, pk, pv, np, pa, L.mv, g->depth, linear,
                                                     window, match, sad, res);
    }
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_temporal_workspace_bytes(void) { return temporal_layout(nullptr).bytes; }

int cga_temporal_predict(const cga_grid *g, const void *d_ref_keys, const uint32_t *d_ref_values,
                         int64_t n_ref, const void *d_pred_keys, const uint32_t *d_pred_values,
                         int64_t n_pred, int window, int max_iter, uint8_t *d_ref_assign,
                         uint8_t *d_pred_assign, double *d_centroids, int32_t *d_mv,
                         int32_t *d_iters, int64_t *d_match, uint32_t *d_sad, int16_t *d_residual,
                         void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || n_ref < 0 || n_pred < 0 || !d_ws) return CGA_EINVAL;
    if (window < 0 || window > kTemporalMaxWindow || max_iter < 1 || max_iter > kTemporalMaxIter)
        return CGA_EINVAL;
    if (n_ref > 0 && (!d_ref_keys || !d_ref_values || !d_ref_assign)) return CGA_EINVAL;
    if (n_pred > 0 && (!d_pred_keys || !d_pred_values || !d_pred_assign || !d_match || !d_sad ||
                       !d_residual))
        return CGA_EINVAL;
    const TemporalLayout L = temporal_layout(d_ws);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(L.ctl, L.st, 2 * sizeof(KmState), nullptr, 0, nullptr, s));
    if (wide_keys(g->depth))
        temporal_launch<uint64_t>(g, (const uint64_t *)d_ref_keys, d_ref_values, n_ref,
                                  (const uint64_t *)d_pred_keys, d_pred_values, n_pred, window,
                                  max_iter, d_ref_assign, d_pred_assign, d_centroids, d_mv, d_iters,
                                  d_match, d_sad, d_residual, L, s);
    else
        temporal_launch<uint32_t>(g, (const uint32_t *)d_ref_keys, d_ref_values, n_ref,
                                  (const uint32_t *)d_pred_keys, d_pred_values, n_pred, window,
                                  max_iter, d_ref_assign, d_pred_assign, d_centroids, d_mv, d_iters,
                                  d_match, d_sad, d_residual, L, s);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
