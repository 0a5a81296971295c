// Attribute payload: the Value array of Section V.
//
// Per-voxel values from per-point ones: every point finds its voxel among the
// CGA's sorted keys by binary search and adds its four 8-bit channels into
// 64-bit per-voxel sums (integer atomics, so the result does not depend on
// their order); a second pass turns sums and point counts into channel
// averages rounded half up, floor((2 sum + count) / (2 count)) -- the colour
// averaging of the grid downsampling in Section III-B.
//
// Values of a merge, Eq. (1): every key of the union looks itself up in both
// inputs; a key in both takes the base cloud's value or the channel average
// of the two (the two choices of Section II-A).
#include "cga_common.h"

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

// acc: 5 words per voxel -- four channel sums, then the point count.
// Consecutive points often share a voxel (a scan line, a dense surface), so
// each wave first sums the runs of equal voxels among its 64 points: the
// point's channels and a count are packed into one word (14 bits per
// channel sum, 64 * 255 < 2^14; the count from bit 56), a wave prefix sum of
// the packed words gives every run's total as a difference, and the last
// lane of a run adds it with at most five atomics.  The sums are integers,
// so the result does not depend on how the points are grouped.
template <typename K>
__global__ __launch_bounds__(256) void k_values_accum(const float *__restrict__ xyz, int64_t n,
                                                      const uint32_t *__restrict__ attr, float o0,
                                                      float o1, float o2, float scale, uint32_t depth,
                                                      bool linear, const K *__restrict__ keys,
                                                      int64_t u_host, const int64_t *d_u,
                                                      unsigned long long *__restrict__ acc,
                                                      uint32_t *err) {
    const int64_t u = dev_count(u_host, d_u) < u_host ? dev_count(u_host, d_u) : u_host;
    const float o[3] = {o0, o1, o2};
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); i0 < n; i0 += stride) {
        const int64_t i = i0 + lane;  // i0 is wave-uniform
        int64_t j = -1;
        uint64_t pv = 0;
        if (i < n) {
            Vox v;
            if (!quantize3(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], o, scale, depth, v)) {
                set_err(err, ERR_NONFINITE);
            } else {
                const uint64_t key = enc3(v.x, v.y, v.z, depth, linear);
                const int64_t f = lower_bound_keys(keys, u, key);
                if (f >= u || (uint64_t)keys[f] != key) {
                    set_err(err, ERR_MISMATCH);
                } else {
                    const uint32_t a = attr[i];
                    j = f;
                    pv = (uint64_t)(a & 0xFFu) | ((uint64_t)((a >> 8) & 0xFFu) << 14) |
                         ((uint64_t)((a >> 16) & 0xFFu) << 28) | ((uint64_t)(a >> 24) << 42) |
                         (1ull << 56);
                }
            }
        }
        const int64_t jp = __shfl_up(j, 1, 64);
        const uint64_t heads = __ballot(lane == 0 || j != jp);
        uint64_t p = pv;  // inclusive prefix sum over the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t t = __shfl_up(p, d, 64);
            if (lane >= d) p += t;
        }
        const uint64_t upto = lane == 63 ? heads : heads & ((2ull << lane) - 1);
        const int start = 63 - __clzll(upto);  // first lane of this lane's run
        const uint64_t before = __shfl(p, start > 0 ? start - 1 : 0, 64);
        const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
        if (tail && j >= 0) {
            const uint64_t sum = p - (start > 0 ? before : 0ull);
            unsigned long long *q = acc + 5 * j;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const unsigned long long w = (sum >> (14 * c)) & 0x3FFFu;
                if (w) atomicAdd(q + c, w);
            }
            atomicAdd(q + 4, (unsigned long long)(sum >> 56));
        }
    }
}

__global__ __launch_bounds__(256) void k_values_final(const unsigned long long *__restrict__ acc,
                                                      int64_t u_host, const int64_t *d_u,
                                                      uint32_t *__restrict__ values, uint32_t *err) {
    const int64_t u = dev_count(u_host, d_u) < u_host ? dev_count(u_host, d_u) : u_host;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < u;
         j += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long *p = acc + 5 * j;
        const uint64_t cnt = p[4];
        if (cnt == 0) {  // a key with no point of this cloud
            set_err(err, ERR_MISMATCH);
            values[j] = 0;
            continue;
        }
        uint32_t v = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) v |= round_half_up(p[c], cnt) << (8 * c);
        values[j] = v;
    }
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

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_voxel_values_workspace_bytes(int64_t u) {
    if (u < 0) return 0;
    Carve c(nullptr);
    c.take<Control>(1);
    c.take<unsigned long long>((size_t)(u > 0 ? u : 1) * 5);
    return c.size();
}

int cga_voxel_values(const cga_grid *g, const float *d_xyz, int64_t n, const uint32_t *d_attr,
                     const void *d_keys, int64_t u, const int64_t *d_u, uint32_t *d_values,
                     void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!grid_valid(g) || n < 0 || u < 0 || !d_ws) return CGA_EINVAL;
    if ((n > 0 && (!d_xyz || !d_attr)) || (u > 0 && (!d_keys || !d_values))) return CGA_EINVAL;
    if (ws_bytes < cga_voxel_values_workspace_bytes(u)) return CGA_EWORKSPACE;
    Carve c(d_ws);
    Control *ctl = c.take<Control>(1);
    unsigned long long *acc = c.take<unsigned long long>((size_t)(u > 0 ? u : 1) * 5);
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(ctl, acc, (size_t)u * 5 * sizeof(unsigned long long), nullptr, 0, nullptr, s));
    const bool linear = g->key_mode == CGA_KEY_LINEAR;
    if (n > 0 && u > 0) {
        CGA_PROF("values_accum", s);
        if (wide_keys(g->depth))
            k_values_accum<uint64_t><<<grid_for(n), 256, 0, s>>>(
                d_xyz, n, d_attr, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth,
                linear, (const uint64_t *)d_keys, u, d_u, acc, &ctl->err);
        else
            k_values_accum<uint32_t><<<grid_for(n), 256, 0, s>>>(
                d_xyz, n, d_attr, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth,
                linear, (const uint32_t *)d_keys, u, d_u, acc, &ctl->err);
    }
    if (u > 0) {
        CGA_PROF("values_final", s);
        k_values_final<<<grid_for(u), 256, 0, s>>>(acc, u, d_u, d_values, &ctl->err);
    }
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
