// Shared device and host helpers of the CGA HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cga.h"

namespace cga {

// ------------------------------------------------------------------ host
extern thread_local int g_last_hip_error;

#define CGA_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) {                                \
            ::cga::g_last_hip_error = (int)e_;                 \
            return CGA_EHIP;                                   \
        }                                                      \
    } while (0)

#define CGA_TRY(expr)              \
    do {                           \
        int r_ = (expr);           \
        if (r_ != CGA_OK) return r_; \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace; every region 256-byte aligned.
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *p) : base((char *)p) {}
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return align_up(off, 256); }
};

bool grid_valid(const cga_grid *g);
inline bool wide_keys(uint32_t depth) { return 3 * depth > 32; }
inline bool wide_keys2(uint32_t depth) { return 2 * depth > 32; }

// Error bits recorded by kernels in the workspace status word.
enum : uint32_t { ERR_NONFINITE = 1u, ERR_CAPACITY = 2u, ERR_MISMATCH = 4u };
int status_from_bits(uint32_t bits);

// Control block at the start of every workspace.
struct Control {
    uint32_t err;           // ERR_* bits of the last call
    uint32_t pad;
    int64_t count;          // output size when the caller gives no d_n_out
    int64_t count2;         // second output size (cga_to_arrays)
    uint32_t tile_ctr[48];  // dynamic tile counters, one per kernel of a call
};
constexpr size_t kControlBytes = 256;
static_assert(sizeof(Control) <= kControlBytes, "control block");

// Enqueue the call prologue: zero the control block, optional regions, and
// set an optional device count output to 0.
int launch_begin(Control *ctl, void *z0, size_t z0_bytes, void *z1, size_t z1_bytes,
                 int64_t *d_n_out, hipStream_t s, int64_t *zero2 = nullptr,
                 int64_t *zero3 = nullptr, int64_t *zero4 = nullptr);
// Synchronise and translate the control block's error bits.
int finish_sync(const Control *ctl, hipStream_t s);

// Optional per-kernel timing.  When enabled (cga_prof_enable), a launch
// whose label matches the filter is bracketed by HIP events recorded on the
// launch's own stream; cga_prof_read waits for them and sums the durations.
struct ProfScope {
    int slot = -1;
    hipStream_t stream = nullptr;
    ProfScope(const char *label, hipStream_t s);
    ~ProfScope();
};
#define CGA_PROF_CAT2(a, b) a##b
#define CGA_PROF_CAT(a, b) CGA_PROF_CAT2(a, b)
#define CGA_PROF(label, s) ::cga::ProfScope CGA_PROF_CAT(prof_scope_, __LINE__)(label, s)

// ---------------------------------------------------------------- device
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Lanes of the wave whose value v has the same low `bits` bits as this
// lane's: per bit, the ballot of the lanes that have it set, flipped where
// this lane has it clear (x ^ 0 or x ^ ~0, the bit's sign extension), and
// any flipped-in difference rules a lane out.
template <int BITS>
__device__ __forceinline__ uint64_t match_low_bits(uint32_t v) {
    uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const int32_t neg = __builtin_amdgcn_sbfe((int32_t)v, b, 1);  // 0 or -1
        const uint64_t bal = __ballot(neg != 0);
        diff_lo |= (uint32_t)bal ^ (uint32_t)neg;
        diff_hi |= (uint32_t)(bal >> 32) ^ (uint32_t)neg;
    }
    return ~(((uint64_t)diff_hi << 32) | diff_lo);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;  // lane 0 -> 0
}

// Agent-scope (whole-GPU, across XCDs) relaxed atomics for chained scans.
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_err(uint32_t *err, uint32_t bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive wave scan (sum) with cross-lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane_id() >= o) v += u;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_max(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane_id() >= o) v = v > u ? v : u;
    }
    return v;
}

// Block-wide exclusive sum of one value per thread.  `s_wave` holds
// BLOCK/64 entries.  Returns the exclusive prefix; *total gets the sum.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_sum(T v, T *s_wave, T *total) {
    constexpr int WAVES = BLOCK / 64;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T inc = wave_incl_sum(v);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    T wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        T x = s_wave[w];
        if (w < wave) wbase += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - v;
}

// Block-wide exclusive max (identity `lo`) of one value per thread.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_max(T v, T lo, T *s_wave, T *total) {
    constexpr int WAVES = BLOCK / 64;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T inc = wave_incl_max(v);
    T exc = __shfl_up(inc, 1, 64);
    if (lane == 0) exc = lo;
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    T wbase = lo, tot = lo;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        T x = s_wave[w];
        if (w < wave) wbase = wbase > x ? wbase : x;
        tot = tot > x ? tot : x;
    }
    __syncthreads();
    *total = tot;
    return wbase > exc ? wbase : exc;
}

// Decoupled look-back (Merrill & Garland 2016) run by one whole wave over a
// window of 64 predecessors: lane l reads the status word of tile t - l, the
// wave finds the nearest inclusive one, and one wave reduction combines every
// value from there to tile t - 1; a walk over m unfinished predecessors costs
// m / 64 round trips instead of m.  Status words carry a 2-bit flag in bits
// 62-63 (0 = not yet published, 1 = aggregate, 2 = inclusive); tiles before
// `first` count as an inclusive zero.  Every lane of the wave must call it;
// every lane gets the result.  Combine is (sum of the low 62 bits).
__device__ __forceinline__ uint64_t lookback_window(const uint64_t *status, int64_t tile,
                                                    int64_t first, uint64_t *nearest_upto) {
    const int lane = lane_id();
    for (;;) {
        const int64_t ti = tile - 1 - lane;
        const uint64_t st = ti >= first ? ld_agent(&status[ti]) : (2ull << 62);
        const uint64_t inc = __ballot((st >> 62) == 2);
        const uint64_t pub = __ballot((st >> 62) != 0);
        // lanes 0 .. f, f the nearest inclusive (every lane when there is none)
        const uint64_t upto = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;
        if ((pub & upto) == upto) {
            *nearest_upto = inc ? upto : 0;
            return st;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__device__ __forceinline__ uint64_t lookback_sum62(const uint64_t *status, int64_t tile,
                                                   int64_t first) {
    const int lane = lane_id();
    uint64_t acc = 0;
    for (int64_t t = tile; ; t -= 64) {
        uint64_t upto;
        const uint64_t st = lookback_window(status, t, first, &upto);
        const uint64_t use = upto ? upto : ~0ull;
        unsigned long long v = ((use >> lane) & 1ull) ? (st & ((1ull << 62) - 1)) : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc += v;
        if (upto) return acc;
    }
}

// Dynamic tile id: tiles are numbered in the order their workgroups start,
// so a tile only ever waits on tiles that are already running.
__device__ __forceinline__ uint32_t next_tile(uint32_t *ctr, uint32_t *s_slot) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(ctr, 1u);
    __syncthreads();
    return *s_slot;
}

__device__ __forceinline__ int64_t dev_count(int64_t n_host, const int64_t *d_n) {
    return d_n ? *d_n : n_host;
}

// ------------------------------------------------------- key bit shuffles
// Spread the low 21 bits of v so bit b lands at bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
// Inverse of spread3: gather bits 3b into bit b.
__device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x1FFFFFull;
    return (uint32_t)v;
}
// Spread the low 32 bits so bit b lands at bit 2b.
__device__ __forceinline__ uint64_t spread2(uint64_t v) {
    v &= 0xFFFFFFFFull;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

struct Vox {
    uint32_t x, y, z;
};

__device__ __forceinline__ uint64_t enc3(uint32_t x, uint32_t y, uint32_t z, uint32_t depth,
                                         bool linear) {
    if (linear)
        return ((uint64_t)x << (2 * depth)) | ((uint64_t)y << depth) | (uint64_t)z;
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__device__ __forceinline__ Vox dec3(uint64_t k, uint32_t depth, bool linear) {
    if (linear) {
        const uint64_t m = (1ull << depth) - 1;
        return Vox{(uint32_t)((k >> (2 * depth)) & m), (uint32_t)((k >> depth) & m),
                   (uint32_t)(k & m)};
    }
    return Vox{compact3(k >> 2), compact3(k >> 1), compact3(k)};
}

// Grid rule: floor(fl32(fl32(p - o) * s)) clamped to [0, 2^d - 1], each
// operation rounded separately (explicit round-to-nearest intrinsics, so no
// contraction into an FMA).  Returns false for a non-finite coordinate.
__device__ __forceinline__ bool quantize3(float px, float py, float pz, const float o[3],
                                          float s, uint32_t depth, Vox &v) {
    const float top = (float)((1u << depth) - 1u);
    const float p[3] = {px, py, pz};
    uint32_t r[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ok = ok && isfinite(p[a]);
        float t = __fsub_rn(p[a], o[a]);
        float u = __fmul_rn(t, s);
        float f = floorf(u);
        f = f >= 0.0f ? f : 0.0f;  // NaN-safe: comparison false -> 0
        f = f <= top ? f : top;
        r[a] = (uint32_t)f;
    }
    v = Vox{r[0], r[1], r[2]};
    return ok;
}

}  // namespace cga
