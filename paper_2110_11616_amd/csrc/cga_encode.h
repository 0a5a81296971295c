// Quantize + encode kernel shared by the build and the Value array: one
// pass over the float32 points writing their keys in input order, with the
// digit histograms of the radix sort that follows accumulated on the side.
#pragma once

#include "cga_common.h"
#include "cga_sort.h"

namespace cga {

constexpr int kEncodeUnroll = 4;

// Quantize + encode one point per thread (grid-stride), with the digit
// histogram of every sort pass accumulated on the side.
template <typename K, int RB>
__global__ __launch_bounds__(256) void k_encode(const float *__restrict__ xyz, int64_t n, float o0,
                                                float o1, float o2, float scale, uint32_t depth,
                                                int linear, K *__restrict__ keys, int passes,
                                                uint32_t *hist, uint32_t *err) {
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_h[];
    __shared__ int s_bad;
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += blockDim.x) s_h[i] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const float o[3] = {o0, o1, o2};
    bool bad = false;
    // kEncodeUnroll points per thread and step, all loaded before any is
    // encoded (more bytes in flight per CU); the wave's points stay
    // consecutive, which the coherent histogram relies on
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 - threadIdx.x < n;
         i0 += kEncodeUnroll * stride) {
        float p[kEncodeUnroll][3];
#pragma unroll
        for (int u = 0; u < kEncodeUnroll; ++u) {
            const int64_t i = i0 + u * stride;
#pragma unroll
            for (int a = 0; a < 3; ++a) p[u][a] = i < n ? xyz[3 * i + a] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kEncodeUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            if (i - threadIdx.x >= n) break;  // block-uniform: no wave of this step has a point
            Vox v;
            const bool ok = quantize3(p[u][0], p[u][1], p[u][2], o, scale, depth, v);
            const K k = (K)enc3(v.x, v.y, v.z, depth, linear != 0);
            if (i < n) {
                bad |= !ok;
                keys[i] = k;
            }
            if (passes && i < n) hist_add_coherent<RB>(s_h, k, passes);
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (passes) hist_flush<RB>(s_h, hist, passes);
    if (threadIdx.x == 0 && s_bad) set_err(err, ERR_NONFINITE);
}

template <typename K, int RB>
inline void encode_launch(const cga_grid *g, const float *xyz, int64_t n, K *keys, int passes,
                          uint32_t *hist, uint32_t *err, hipStream_t s) {
    int64_t blocks = (n + 256 * 8 - 1) / (256 * 8);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    CGA_PROF("encode", s);
    k_encode<K, RB><<<(unsigned)blocks, 256, hist_lds_bytes(passes, RB), s>>>(
        xyz, n, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth,
        g->key_mode == CGA_KEY_LINEAR, keys, passes, hist, err);
}

template <typename K>
inline void encode_dispatch(const cga_grid *g, const float *xyz, int64_t n, K *keys, int rb,
                            int passes, uint32_t *hist, uint32_t *err, hipStream_t s) {
    switch (rb) {
        case 4: encode_launch<K, 4>(g, xyz, n, keys, passes, hist, err, s); break;
        case 5: encode_launch<K, 5>(g, xyz, n, keys, passes, hist, err, s); break;
        case 6: encode_launch<K, 6>(g, xyz, n, keys, passes, hist, err, s); break;
        case 7: encode_launch<K, 7>(g, xyz, n, keys, passes, hist, err, s); break;
        case 9: encode_launch<K, 9>(g, xyz, n, keys, passes, hist, err, s); break;
        case 10: encode_launch<K, 10>(g, xyz, n, keys, passes, hist, err, s); break;
        case 11: encode_launch<K, 11>(g, xyz, n, keys, passes, hist, err, s); break;
        default: encode_launch<K, 8>(g, xyz, n, keys, passes, hist, err, s); break;
    }
}

}  // namespace cga
