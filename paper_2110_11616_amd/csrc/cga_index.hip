// Learned index over a sorted unique uint64 key array: a two-stage model of
// the key -> rank function (fp64 root router, linear or piecewise linear,
// per-leaf fp32 linear or 1-16-1 ReLU network), per-leaf max-error windows,
// and a verified last-mile lookup with binary-search fallback, so that every
// result equals the plain lower bound for any sorted key array.  Trained on the GPU by the kernels below: fp64 sums
// for the least-squares fits, a full-batch forward/backward pass plus Adam
// per network leaf (one workgroup per leaf, fixed reduction order, so
// training is deterministic).
//
// Every float expression that decides a rank is written with explicit
// round-to-nearest intrinsics (fmaf, __fmul_rn, ...), so window building and
// lookups evaluate bit-identical predictions.
#include "cga_common.h"

namespace cga {

constexpr uint32_t kIndexMagic = 0x49414743u;  // "CGAI"
constexpr uint32_t kIndexVersion = 3;
constexpr int kMlpHidden = 16;
constexpr int kMlpParams = 3 * kMlpHidden + 1;  // w1[16], b1[16], w2[16], b2
constexpr int kLeafBlock = 64;  // one wave per leaf
// Leaf count limit.  Routing computes the leaf id in fp64 (exact far beyond
// this); the limit keeps the leaf records within 1 GiB (linear) or 4 GiB
// (network) and a leaf's int32 window arithmetic far from overflow.
constexpr uint32_t kMaxLeaves = 1u << 24;
// Keys at evenly spaced ranks kept in the index as its key fingerprint: a
// lookup compares the given array at those ranks (CGA_EMISMATCH on a
// difference).
constexpr uint32_t kIndexSamples = 4096;
constexpr int kLeafCache = 1024;  // leaf inputs kept in LDS (floats)
constexpr int kMlpBatch = 512;    // training samples per network leaf and epoch
constexpr int kMlpPad = 64;       // gradient vector length for the halving reduction

struct IndexHeader {
    uint32_t magic, version, n_leaves, leaf_kind;
    int64_t n;
    uint64_t kmin, kmax;
    double root_a, root_b, inv_span;  // root model and input scale (fp64)
    uint32_t nparams;
    uint32_t root_segs;
    uint32_t leaf_stride;  // bytes per leaf record
    uint32_t nsamples;     // fingerprint keys: min(n, kIndexSamples)
};
static_assert(sizeof(IndexHeader) <= 256, "index header");

// One leaf = one record: this head, then its parameters; 64 bytes for a
// linear leaf, 256 for a network leaf, so a lookup reads one or a few lines.
struct LeafHead {
    int64_t first;    // first rank of the leaf
    uint64_t kfirst;  // key at that rank
    int32_t count;    // keys in the leaf
    float isp;        // 1 / (last key - first key), or 0
    int32_t err_lo, err_hi;
};
static_assert(sizeof(LeafHead) == 32, "leaf head");

// One root segment: input at its start, output at its start and end, slope
// (fp64: a float input would give every key in one 2^-24 step of the key
// range the same leaf, and the keys of a dense cluster share such steps).
struct RootSeg {
    double x0, y0, y1, slope;
};

__host__ __device__ inline size_t idx_align(size_t v) { return (v + 255) / 256 * 256; }
__host__ __device__ inline uint32_t leaf_stride(uint32_t nparams) {
    return nparams <= 8 ? 64u : 256u;
}

struct IndexView {
    IndexHeader *h;
    double *rx;     // R segment start inputs (searched)
    RootSeg *seg;   // R segments
    uint64_t *samp; // fingerprint: the keys at ranks sample_rank(s)
    char *leaves;   // n_leaves records of leaf_stride bytes
    __device__ LeafHead &head(uint32_t j) const { return *(LeafHead *)(leaves + (size_t)j * h->leaf_stride); }
    __device__ float *params(uint32_t j) const {
        return (float *)(leaves + (size_t)j * h->leaf_stride + sizeof(LeafHead));
    }
};

__host__ __device__ inline size_t index_layout(char *base, uint32_t L, uint32_t nparams,
                                               uint32_t R, IndexView *v) {
    size_t off = 256;
    IndexView w;
    w.h = (IndexHeader *)base;
    w.rx = base ? (double *)(base + off) : nullptr;
    off = idx_align(off + (size_t)R * sizeof(double));
    w.seg = base ? (RootSeg *)(base + off) : nullptr;
    off = idx_align(off + (size_t)R * sizeof(RootSeg));
    w.samp = base ? (uint64_t *)(base + off) : nullptr;
    off = idx_align(off + (size_t)kIndexSamples * sizeof(uint64_t));
    w.leaves = base ? base + off : nullptr;
    off = idx_align(off + (size_t)L * leaf_stride(nparams));
    if (v) *v = w;
    return off;
}

// Rank of fingerprint key s of m (m = min(n, kIndexSamples)): evenly spaced
// over [0, n - 1], both ends included.
__host__ __device__ inline int64_t sample_rank(uint32_t s, uint32_t m, int64_t n) {
    return m > 1 ? (int64_t)(((uint64_t)s * (uint64_t)(n - 1)) / (m - 1)) : 0;
}

// ------------------------------------------------------------- model maths
// Root input: the key's offset in the array's key range, scaled to [0, 1].
__device__ __forceinline__ double root_x(uint64_t q, uint64_t kmin, uint64_t kmax, double isp) {
    const uint64_t c = q <= kmin ? 0ull : (q >= kmax ? kmax - kmin : q - kmin);
    return __dmul_rn((double)c, isp);
}

// Root routing; monotone in q.  A piecewise-linear root evaluates segment s
// (the last segment whose start input is <= x) clamped to its end values,
// so adjacent segments cannot overlap after rounding.  The segment search
// runs over `rx`, every `stride`-th segment start (`nrx` of them, possibly an
// LDS copy), then over the at most `stride` starts of that block in the
// index; stride 1 searches the index's starts alone.
__device__ __forceinline__ uint32_t route(const IndexHeader &h, const IndexView &v, const double *rx,
                                          uint32_t stride, uint32_t nrx, uint64_t q) {
    const double x = root_x(q, h.kmin, h.kmax, h.inv_span);
    double y;
    if (h.root_segs == 0) {
        y = fma(h.root_a, x, h.root_b);
    } else {
        uint32_t lo = 0, len = nrx;  // last i with rx[i] <= x (rx[0] = 0)
        while (len > 1) {
            const uint32_t half = len >> 1;
            lo = rx[lo + half] <= x ? lo + half : lo;
            len -= half;
        }
        if (stride > 1) {
            lo *= stride;
            len = h.root_segs - lo < stride ? h.root_segs - lo : stride;
            while (len > 1) {
                const uint32_t half = len >> 1;
                lo = v.rx[lo + half] <= x ? lo + half : lo;
                len -= half;
            }
        }
        const RootSeg g = v.seg[lo];
        y = fma(g.slope, __dsub_rn(x, g.x0), g.y0);
        y = y >= g.y0 ? (y <= g.y1 ? y : g.y1) : g.y0;
    }
    y = floor(y);
    const double top = (double)(h.n_leaves - 1);
    const double c = y >= 0.0 ? (y <= top ? y : top) : 0.0;  // NaN -> 0
    return (uint32_t)c;
}

__device__ __forceinline__ float mlp_forward(const float *p, float x) {
    float f = p[3 * kMlpHidden];
#pragma unroll
    for (int h = 0; h < kMlpHidden; ++h) {
        const float z = fmaf(p[h], x, p[kMlpHidden + h]);
        f = fmaf(p[2 * kMlpHidden + h], fmaxf(z, 0.0f), f);
    }
    return f;
}

// Leaf range [f0, f1) clamped to [0, n], and the predicted rank in [f0, f1].
__device__ __forceinline__ int64_t leaf_predict(const LeafHead &lh, const float *p, uint32_t kind,
                                                uint64_t q, int64_t n, int64_t *f0o, int64_t *f1o) {
    int64_t f0 = lh.first, nj = lh.count;
    f0 = f0 < 0 ? 0 : (f0 > n ? n : f0);
    nj = nj < 0 ? 0 : (nj > n - f0 ? n - f0 : nj);
    *f0o = f0;
    *f1o = f0 + nj;
    const float x = q <= lh.kfirst ? 0.0f : __fmul_rn((float)(q - lh.kfirst), lh.isp);
    const float f = kind == 0 ? fmaf(p[0], x, p[1]) : mlp_forward(p, x);
    float r = rintf(__fmul_rn((float)nj, f));
    r = r >= 0.0f ? r : 0.0f;  // NaN -> 0
    const float fnj = (float)nj;
    r = r <= fnj ? r : fnj;
    int64_t ri = (int64_t)r;
    ri = ri > nj ? nj : ri;
    return f0 + ri;
}

// Sample s of a network leaf sits at LDS slot s + s / 16, so that the lanes'
// runs of up to 8 consecutive samples mostly start in different banks.
constexpr int kMlpSlots = kMlpBatch + kMlpBatch / 16 + 1;
__device__ __forceinline__ int lds_pad(int s) { return s + (s >> 4); }

// Inclusive wave-wide prefix sum by DPP row shifts (within rows of 16 lanes)
// and row broadcasts (across rows); lanes without a source add zero.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_shift(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, kRowMask, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, kRowMask, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double wave_prefix_sum(double v) {
    v += dpp_shift<0x111, 0xf>(v);  // row_shr:1
    v += dpp_shift<0x112, 0xf>(v);  // row_shr:2
    v += dpp_shift<0x114, 0xf>(v);  // row_shr:4
    v += dpp_shift<0x118, 0xf>(v);  // row_shr:8
    v += dpp_shift<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_shift<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Gradient of the summed squared error of one 1-16-1 network over m <= kMlpBatch
// samples (sx ascending, st; slots lds_pad(s)) held in LDS, for parameter
// c = lane (w1, b1, w2, b2 order; 0 for the padding lanes).  Hidden unit h is
// active where fmaf(w1_h, x, b1_h) > 0; that is monotone in x, so over
// ascending samples the active set is one contiguous run [a0, a1).  With
// dr_s = 2 (f(x_s) - t_s) every gradient is a sum of dr_s or dr_s x_s over
// that run:
//   dE/dw1_h = w2_h sum dr x,  dE/db1_h = w2_h sum dr,
//   dE/dw2_h = sum dr (w1_h x + b1_h) = w1_h sum dr x + b1_h sum dr,
//   dE/db2 = sum dr over all samples,
// so after one forward pass (lane L takes the consecutive samples
// [L per, L per + per)) the wave builds the two prefix sums and each lane
// finds its unit's run by a binary search.  A prefix sum up to sample s is
// the fp64 total of the lanes before s's lane (e0 / e1, one per lane) plus
// the fp32 running sum of at most 8 terms inside that lane (l0 / l1, one per
// sample), which keeps the LDS of a leaf small enough for four waves per
// SIMD.  The lane also returns its samples' unscaled loss, sum (f - t)^2.
// One wave; the wave must be converged.  kPer >= per: the samples a lane
// evaluates (those past its run count zero).
template <int kPer>
__device__ __forceinline__ double mlp_grad_sorted(const float *sp, const float *sx, const float *st,
                                                  int m, float *l0, float *l1, double *e0s,
                                                  double *e1s, int lane, double *loss) {
    float p[kMlpParams];
#pragma unroll
    for (int c = 0; c < kMlpParams; ++c) p[c] = sp[c];
    const int per = (m + 63) >> 6;
    const int s0 = lane * per < m ? lane * per : m;
    const int cnt = s0 + per < m ? per : m - s0;
    double pre0[kPer], pre1[kPer], r0 = 0.0, r1 = 0.0, l2 = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        // every lane evaluates kPer samples (independent chains the compiler
        // can interleave); those past its run count zero
        const int si = s0 + i < m ? s0 + i : (m > 0 ? m - 1 : 0);
        const float x = sx[lds_pad(si)];
        const double r = i < cnt ? (double)__fsub_rn(mlp_forward(p, x), st[lds_pad(si)]) : 0.0;
        l2 += r * r;
        r0 += 2.0 * r;
        r1 += (2.0 * r) * (i < cnt ? (double)x : 0.0);
        pre0[i] = r0;
        pre1[i] = r1;
    }
    e0s[lane] = wave_prefix_sum(r0) - r0;  // exclusive
    e1s[lane] = wave_prefix_sum(r1) - r1;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
        if (i < cnt) {
            l0[lds_pad(s0 + i)] = (float)pre0[i];
            l1[lds_pad(s0 + i)] = (float)pre1[i];
        }
    __syncthreads();
    *loss = l2;
    // sums of dr and dr x over the samples before a (0 <= a <= m)
    auto prefix = [&](int a, double &p0, double &p1) {
        if (a == 0) {
            p0 = p1 = 0.0;
            return;
        }
        const int sl = a - 1, L = sl / per;
        p0 = e0s[L] + (double)l0[lds_pad(sl)];
        p1 = e1s[L] + (double)l1[lds_pad(sl)];
    };
    if (lane == 3 * kMlpHidden) {
        double t0, t1;
        prefix(m, t0, t1);
        return t0;
    }
    if (lane > 3 * kMlpHidden) return 0.0;
    const int h = lane & (kMlpHidden - 1);
    const float w = sp[h], b = sp[kMlpHidden + h], w2 = sp[2 * kMlpHidden + h];
    // the samples where activity differs from `up` form a prefix: inactive
    // ones before an ascending run, active ones before a descending one
    const bool up = w > 0.0f;
    int lo = 0, len = m;
    while (len > 0) {
        const int half = len >> 1;
        if ((fmaf(w, sx[lds_pad(lo + half)], b) > 0.0f) != up) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    const int a0 = up ? lo : 0, a1 = up ? m : lo;
    double p00, p01, p10, p11;
    prefix(a0, p00, p01);
    prefix(a1, p10, p11);
    const double S0 = p10 - p00, S1 = p11 - p01;
    if (lane < kMlpHidden) return (double)w2 * S1;
    if (lane < 2 * kMlpHidden) return (double)w2 * S0;
    return (double)w * S1 + (double)b * S0;
}

// mlp_grad_sorted with the fewest samples per lane that hold m (<= kMlpBatch).
__device__ __forceinline__ double mlp_grad(const float *sp, const float *sx, const float *st, int m,
                                           float *l0, float *l1, double *e0s, double *e1s,
                                           int lane, double *loss) {
    if (m <= 64) return mlp_grad_sorted<1>(sp, sx, st, m, l0, l1, e0s, e1s, lane, loss);
    if (m <= 128) return mlp_grad_sorted<2>(sp, sx, st, m, l0, l1, e0s, e1s, lane, loss);
    if (m <= 256) return mlp_grad_sorted<4>(sp, sx, st, m, l0, l1, e0s, e1s, lane, loss);
    return mlp_grad_sorted<kMlpBatch / 64>(sp, sx, st, m, l0, l1, e0s, e1s, lane, loss);
}

// ----------------------------------------------------------------- kernels
__global__ void k_index_header(const uint64_t *keys, int64_t n, uint32_t L, uint32_t kind,
                               uint32_t np, uint32_t R, IndexHeader *h) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    h->root_segs = R;
    h->leaf_stride = leaf_stride(np);
    h->magic = kIndexMagic;
    h->version = kIndexVersion;
    h->n_leaves = L;
    h->leaf_kind = kind;
    h->nparams = np;
    h->n = n;
    h->nsamples = n < (int64_t)kIndexSamples ? (uint32_t)n : kIndexSamples;
    h->kmin = n > 0 ? keys[0] : 0;
    h->kmax = n > 0 ? keys[n - 1] : 0;
    const uint64_t span = h->kmax - h->kmin;
    h->inv_span = span ? __ddiv_rn(1.0, (double)span) : 0.0;
    h->root_a = (double)L;  // provisional (k_root_final overwrites)
    h->root_b = 0.0;
}

// The fingerprint: keys at nsamples evenly spaced ranks.
__global__ void k_index_samples(const uint64_t *__restrict__ keys, int64_t n, char *index) {
    const IndexHeader &h = *(const IndexHeader *)index;
    IndexView v;
    index_layout(index, h.n_leaves, h.nparams, h.root_segs, &v);
    const uint32_t m = h.nsamples;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < m; s += gridDim.x * blockDim.x)
        v.samp[s] = keys[sample_rank(s, m, n)];
}

// Partial least-squares sums of y = rank * L / n on x (fp64).
__global__ __launch_bounds__(256) void k_root_partial(const uint64_t *__restrict__ keys, int64_t n,
                                                      const IndexHeader *h, double *partial) {
    __shared__ double s[4][256];
    const uint64_t kmin = h->kmin, kmax = h->kmax;
    const double isp = h->inv_span;
    const double scale = (double)h->n_leaves / (double)n;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)root_x(keys[i], kmin, kmax, isp);
        const double y = (double)i * scale;
        sx += x;
        sy += y;
        sxx += x * x;
        sxy += x * y;
    }
    s[0][threadIdx.x] = sx;
    s[1][threadIdx.x] = sy;
    s[2][threadIdx.x] = sxx;
    s[3][threadIdx.x] = sxy;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

// Least-squares line from the block partials, summed in a fixed order (each
// thread a strided subset, then a tree), so the fit is deterministic.
__global__ __launch_bounds__(256) void k_root_final(const double *partial, int blocks, int64_t n,
                                                    IndexHeader *h) {
    __shared__ double s[4][256];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < blocks; b += 256)
        for (int c = 0; c < 4; ++c) acc[c] += partial[4 * b + c];
    for (int c = 0; c < 4; ++c) s[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sx = s[0][0], sy = s[1][0], sxx = s[2][0], sxy = s[3][0];
    const double dn = (double)n;
    const double den = dn * sxx - sx * sx;
    double a = den != 0.0 ? (dn * sxy - sx * sy) / den : 0.0;
    double b = (sy - a * sx) / dn;
    if (!(a > 0.0) || !isfinite(a) || !isfinite(b)) {
        a = (double)h->n_leaves;  // degenerate fit: split the key range evenly
        b = 0.0;
    }
    h->root_a = a;
    h->root_b = b;
}

// Piecewise-linear root: segment t runs between the keys at ranks
// t * (n - 1) / R and (t + 1) * (n - 1) / R.
__global__ void k_root_knots(const uint64_t *__restrict__ keys, int64_t n, char *index) {
    const IndexHeader &h = *(const IndexHeader *)index;
    IndexView v;
    index_layout(index, h.n_leaves, h.nparams, h.root_segs, &v);
    const uint32_t R = h.root_segs;
    const double fl = (double)h.n_leaves, fn = (double)n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < R; t += gridDim.x * blockDim.x) {
        const int64_t r0 = (int64_t)(((uint64_t)t * (uint64_t)(n - 1)) / R);
        const int64_t r1 = (int64_t)(((uint64_t)(t + 1) * (uint64_t)(n - 1)) / R);
        const double x0 = t == 0 ? 0.0 : root_x(keys[r0], h.kmin, h.kmax, h.inv_span);
        const double x1 = root_x(keys[r1], h.kmin, h.kmax, h.inv_span);
        RootSeg g;
        g.x0 = x0;
        g.y0 = __ddiv_rn(__dmul_rn((double)r0, fl), fn);
        g.y1 = __ddiv_rn(__dmul_rn((double)r1, fl), fn);
        const double dx = __dsub_rn(x1, x0);
        g.slope = dx > 0.0 ? __ddiv_rn(__dsub_rn(g.y1, g.y0), dx) : 0.0;
        v.seg[t] = g;
        v.rx[t] = x0;
    }
}

// first[j] = first rank routed to a leaf >= j (routing is monotone), so leaf j
// holds ranks [first[j], first[j + 1]); first[L] = n.  Three passes, each
// parallel over keys or leaves (an empty leaf takes the next non-empty
// leaf's first rank, whatever the run of empty leaves):
//   1. every entry to n;
//   2. the first key of every run of equal leaf ids writes its rank there;
//   3. suffix minimum over the L + 1 entries, in tiles of kFirstTile.
constexpr int kFirstBlock = 1024;
constexpr int kFirstItems = 4;
constexpr int kFirstTile = kFirstBlock * kFirstItems;

__global__ __launch_bounds__(256) void k_leaf_first_fill(int64_t *first, int64_t count, int64_t v) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
         j += (int64_t)gridDim.x * blockDim.x)
        first[j] = v;
}

__global__ __launch_bounds__(256) void k_leaf_first_scatter(const uint64_t *__restrict__ keys,
                                                            int64_t n, const char *index,
                                                            int64_t *first) {
    IndexView v;
    const IndexHeader &h = *(const IndexHeader *)index;
    index_layout((char *)index, h.n_leaves, h.nparams, h.root_segs, &v);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t lj = route(h, v, v.rx, 1, h.root_segs, keys[i]);
        if (i == 0 || route(h, v, v.rx, 1, h.root_segs, keys[i - 1]) != lj) first[lj] = i;
    }
}

// Minimum of each tile of first[0 .. count).
__global__ __launch_bounds__(kFirstBlock) void k_leaf_first_tiles(const int64_t *first,
                                                                  int64_t count, int64_t *tile_min) {
    __shared__ int64_t s_w[kFirstBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kFirstTile;
    int64_t m = INT64_MAX;
    for (int u = 0; u < kFirstItems; ++u) {
        const int64_t j = base + (int64_t)threadIdx.x * kFirstItems + u;
        if (j < count) m = first[j] < m ? first[j] : m;
    }
    int64_t tot;
    block_excl_max<kFirstBlock, int64_t>(-(m == INT64_MAX ? INT64_MAX - 1 : m), INT64_MIN, s_w, &tot);
    if (threadIdx.x == 0) tile_min[blockIdx.x] = -tot;
}

// In-place suffix minimum: each tile combines the minimum of the tiles after
// it (a block reduction over tile_min) with its own entries, scanned from
// the end (thread t holds the t-th group of kFirstItems entries counted from
// the tile's end; an exclusive prefix max of the negated group minima over
// the threads gives each group the minimum of the entries after it).
__global__ __launch_bounds__(kFirstBlock) void k_leaf_first_suffix(int64_t *first, int64_t count,
                                                                   const int64_t *tile_min,
                                                                   int64_t tiles) {
    __shared__ int64_t s_w[kFirstBlock / 64];
    const int64_t t = blockIdx.x;
    int64_t later = INT64_MAX;
    for (int64_t u = t + 1 + threadIdx.x; u < tiles; u += kFirstBlock)
        later = tile_min[u] < later ? tile_min[u] : later;
    int64_t tot;
    block_excl_max<kFirstBlock, int64_t>(-(later == INT64_MAX ? INT64_MAX - 1 : later), INT64_MIN,
                                         s_w, &tot);
    later = -tot;  // minimum over every later tile (INT64_MAX - 1 when none)
    const int64_t base = t * kFirstTile;
    const int64_t g0 = base + kFirstTile - (int64_t)(threadIdx.x + 1) * kFirstItems;  // group start
    int64_t e[kFirstItems];
    int64_t gm = INT64_MAX - 1;
    for (int u = 0; u < kFirstItems; ++u) {
        const int64_t j = g0 + u;
        e[u] = j < count ? first[j] : INT64_MAX - 1;
        gm = e[u] < gm ? e[u] : gm;
    }
    const int64_t ex = block_excl_max<kFirstBlock, int64_t>(-gm, INT64_MIN, s_w, &tot);
    int64_t run = ex == INT64_MIN ? INT64_MAX - 1 : -ex;  // minimum of the tile's later groups
    run = later < run ? later : run;
    for (int u = kFirstItems - 1; u >= 0; --u) {
        run = e[u] < run ? e[u] : run;
        const int64_t j = g0 + u;
        if (j < count) first[j] = run;
    }
}

// Linear leaves, one wave per leaf: least-squares fit, leaf record, window
// reset.
__global__ __launch_bounds__(kLeafBlock) void k_leaf_fit_linear(const uint64_t *__restrict__ keys,
                                                                char *index, const int64_t *first) {
    __shared__ float s_x[kLeafCache];

    IndexView v;
    const IndexHeader &h = *(const IndexHeader *)index;
    index_layout(index, h.n_leaves, h.nparams, h.root_segs, &v);
    const uint32_t j = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t f0 = first[j], f1 = first[j + 1], nj = f1 - f0;
    LeafHead &lh = v.head(j);
    float *par = v.params(j);
    if (nj <= 0) {
        if (tid == 0) {
            lh.first = f0;
            lh.kfirst = 0;
            lh.count = 0;
            lh.isp = 0.0f;
            lh.err_lo = 0;
            lh.err_hi = 0;
        }
        for (uint32_t c = tid; c < h.nparams; c += blockDim.x) par[c] = 0.0f;
        return;
    }
    const uint64_t kf = keys[f0];
    const uint64_t span = keys[f1 - 1] - kf;
    const float isp = span ? __fdiv_rn(1.0f, (float)span) : 0.0f;
    auto xof = [&](int64_t s) -> float {
        return s < kLeafCache ? s_x[s] : __fmul_rn((float)(keys[f0 + s] - kf), isp);
    };
    for (int64_t s = tid; s < nj && s < kLeafCache; s += blockDim.x)
        s_x[s] = __fmul_rn((float)(keys[f0 + s] - kf), isp);
    if (tid == 0) {
        lh.first = f0;
        lh.kfirst = kf;
        lh.count = (int32_t)nj;
        lh.isp = isp;
        lh.err_lo = 0x7FFFFFFF;
        lh.err_hi = (int32_t)0x80000000;
    }
    __syncthreads();

    {
        // least squares of t = s / n_j on x (fp64 sums)
        double acc[4] = {0, 0, 0, 0};
        for (int64_t s = tid; s < nj; s += blockDim.x) {
            const double x = (double)xof(s), t = (double)s / (double)nj;
            acc[0] += x;
            acc[1] += t;
            acc[2] += x * x;
            acc[3] += x * t;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
        if (tid == 0) {
            const double dn = (double)nj;
            const double den = dn * acc[2] - acc[0] * acc[0];
            const double a = den > 0.0 ? (dn * acc[3] - acc[0] * acc[1]) / den : 0.0;
            const double b = (acc[1] - a * acc[0]) / dn;
            par[0] = (float)a;
            par[1] = (float)b;
        }
    }
}

// Full-batch Adam on the network in s_p (lane c owns parameter c and its
// moments) for `epochs` epochs over the m samples in LDS.
template <int kPer>
__device__ __forceinline__ void mlp_adam(float *s_p, const float *s_x, const float *s_t, int m,
                                         float *s_l0, float *s_l1, double *s_e0, double *s_e1,
                                         int tid, uint32_t epochs, float lr) {
    const float b1c = 0.9f, b2c = 0.999f, eps = 1e-8f;
    const double dm = (double)m;
    float pw1 = 1.0f, pw2 = 1.0f;  // b1c^t, b2c^t
    float own = s_p[tid], am = 0.0f, av = 0.0f;
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        double loss;
        const double gsum =
            mlp_grad_sorted<kPer>(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, &loss);
        pw1 = __fmul_rn(pw1, b1c);
        pw2 = __fmul_rn(pw2, b2c);
        __syncthreads();  // every lane has read this epoch's parameters and sums
        if (tid < kMlpParams) {
            const float gr = (float)(gsum / dm);
            am = fmaf(b1c, am, __fmul_rn(1.0f - b1c, gr));
            av = fmaf(b2c, av, __fmul_rn(__fmul_rn(1.0f - b2c, gr), gr));
            const float mh = __fdiv_rn(am, 1.0f - pw1), vh = __fdiv_rn(av, 1.0f - pw2);
            own = __fsub_rn(own, __fdiv_rn(__fmul_rn(lr, mh), __fadd_rn(sqrtf(vh), eps)));
            s_p[tid] = own;
        }
        __syncthreads();
    }
}

// Network leaves, one wave per leaf: initialise the 1-16-1 network as the
// piecewise-linear interpolant of the leaf's key -> rank map at 17 rank
// quantiles, then train it with full-batch Adam on the mean squared error.
// A leaf of more than kMlpBatch keys trains on kMlpBatch of them spaced
// evenly by rank (its window is still measured over every key).  The
// samples ascend, so per epoch one forward pass and two prefix sums give lane
// c the gradient for parameter c (mlp_grad_sorted), which it updates with its
// own Adam moments and publishes through LDS.
__global__ __launch_bounds__(kLeafBlock) void k_leaf_fit_mlp(const uint64_t *__restrict__ keys,
                                                             char *index, const int64_t *first,
                                                             uint32_t epochs, float lr) {
    __shared__ float s_x[kMlpSlots], s_t[kMlpSlots], s_l0[kMlpSlots], s_l1[kMlpSlots];
    __shared__ double s_e0[64], s_e1[64];
    __shared__ float s_p[kMlpPad];
    float *const s_kx = s_l0, *const s_kt = s_l1;  // initial knots, before the first epoch
    IndexView v;
    const IndexHeader &h = *(const IndexHeader *)index;
    index_layout(index, h.n_leaves, h.nparams, h.root_segs, &v);
    const uint32_t j = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t f0 = first[j], f1 = first[j + 1], nj = f1 - f0;
    LeafHead &lh = v.head(j);
    float *par = v.params(j);
    if (nj <= 0) {  // block-uniform
        if (tid == 0) {
            lh.first = f0;
            lh.kfirst = 0;
            lh.count = 0;
            lh.isp = 0.0f;
            lh.err_lo = 0;
            lh.err_hi = 0;
        }
        for (uint32_t c = tid; c < h.nparams; c += blockDim.x) par[c] = 0.0f;
        return;
    }
    const uint64_t kf = keys[f0];
    const uint64_t span = keys[f1 - 1] - kf;
    const float isp = span ? __fdiv_rn(1.0f, (float)span) : 0.0f;
    const float fnj = (float)nj;
    const int m = nj < kMlpBatch ? (int)nj : kMlpBatch;  // samples per epoch
    for (int i = tid; i < m; i += kLeafBlock) {
        const int64_t r = m == nj ? i : ((int64_t)i * nj) / m;  // < 2^41
        s_x[lds_pad(i)] = __fmul_rn((float)(keys[f0 + r] - kf), isp);
        s_t[lds_pad(i)] = __fdiv_rn((float)r, fnj);
    }
    if (tid <= kMlpHidden) {
        const int64_t r = ((int64_t)tid * (nj - 1)) / kMlpHidden;  // < 2^35
        s_kx[tid] = __fmul_rn((float)(keys[f0 + r] - kf), isp);
        s_kt[tid] = __fdiv_rn((float)r, fnj);
    }
    if (tid == 0) {
        lh.first = f0;
        lh.kfirst = kf;
        lh.count = (int32_t)nj;
        lh.isp = isp;
        lh.err_lo = 0x7FFFFFFF;
        lh.err_hi = (int32_t)0x80000000;
    }
    __syncthreads();
    if (tid == 0) {
        float prev = 0.0f;
        for (int q = 0; q < kMlpHidden; ++q) {
            const float dx = __fsub_rn(s_kx[q + 1], s_kx[q]);
            const float sl = dx > 0.0f ? __fdiv_rn(__fsub_rn(s_kt[q + 1], s_kt[q]), dx) : 0.0f;
            s_p[q] = 1.0f;                                  // w1
            s_p[kMlpHidden + q] = -s_kx[q];                 // b1
            s_p[2 * kMlpHidden + q] = __fsub_rn(sl, prev);  // w2: change of slope
            prev = sl;
        }
        s_p[3 * kMlpHidden] = s_kt[0];  // b2
        for (int c = kMlpParams; c < kMlpPad; ++c) s_p[c] = 0.0f;
    }
    __syncthreads();

    // the epoch loop at the fewest samples per lane that hold m
    if (m <= 64) mlp_adam<1>(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, epochs, lr);
    else if (m <= 128) mlp_adam<2>(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, epochs, lr);
    else if (m <= 256) mlp_adam<4>(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, epochs, lr);
    else mlp_adam<kMlpBatch / 64>(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, epochs, lr);
    for (uint32_t c = tid; c < h.nparams; c += blockDim.x) par[c] = c < (uint32_t)kMlpParams ? s_p[c] : 0.0f;
}

// Window of every leaf: min / max of (rank - predicted rank) over its keys.
// Keys are sorted and routing is monotone, so a wave's 64 keys usually fall
// in one leaf; such a wave reduces first and updates the leaf once.
__global__ __launch_bounds__(256) void k_leaf_err(const uint64_t *__restrict__ keys, int64_t n,
                                                  char *index) {
    IndexView v;
    const IndexHeader &h = *(const IndexHeader *)index;
    index_layout(index, h.n_leaves, h.nparams, h.root_segs, &v);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); i0 < n; i0 += stride) {
        const int64_t i = i0 + lane;  // i0 is wave-uniform, so lane 0 is always in range
        const bool valid = i < n;
        uint32_t j = 0xFFFFFFFFu;
        int32_t ec = 0;
        if (valid) {
            const uint64_t q = keys[i];
            j = route(h, v, v.rx, 1, h.root_segs, q);
            int64_t f0, f1;
            const int64_t e = i - leaf_predict(v.head(j), v.params(j), h.leaf_kind, q, n, &f0, &f1);
            ec = (int32_t)(e > 0x3FFFFFFF ? 0x3FFFFFFF : (e < -0x3FFFFFFF ? -0x3FFFFFFF : e));
        }
        const uint32_t j0 = __shfl(j, 0, 64);
        if (__ballot(valid && j == j0) == __ballot(valid)) {
            int32_t lo = valid ? ec : 0x7FFFFFFF, hi = valid ? ec : (int32_t)0x80000000;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int32_t a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
                lo = a < lo ? a : lo;
                hi = b > hi ? b : hi;
            }
            if (lane == 0) {
                LeafHead &lh = v.head(j0);
                atomicMin(&lh.err_lo, lo);
                atomicMax(&lh.err_hi, hi);
            }
        } else if (valid) {
            LeafHead &lh = v.head(j);
            atomicMin(&lh.err_lo, ec);
            atomicMax(&lh.err_hi, ec);
        }
    }
}

template <typename K>
__device__ __forceinline__ int64_t lb_range(const K *keys, int64_t lo, int64_t hi, K q) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int kLookupBlock = 1024;
constexpr uint32_t kLdsSegs = 4096;  // root segment starts staged in LDS up to this many

__global__ __launch_bounds__(kLookupBlock) void k_index_lookup(
    const char *__restrict__ index, const uint64_t *__restrict__ keys, int64_t n,
    const uint64_t *__restrict__ q, int64_t nq, int64_t *__restrict__ rank,
    uint8_t *__restrict__ found, unsigned long long *fallbacks, uint32_t *err) {
    __shared__ double s_rx[kLdsSegs];
    const IndexHeader h = *(const IndexHeader *)index;
    const bool ok = h.magic == kIndexMagic && h.version == kIndexVersion && h.n == n &&
                    h.n_leaves >= 1 && h.n_leaves <= kMaxLeaves && h.leaf_kind <= 1 &&
                    h.nparams == (h.leaf_kind ? (uint32_t)kMlpParams : 2u) &&
                    h.root_segs <= 65536 && h.leaf_stride == leaf_stride(h.nparams) &&
                    h.nsamples == (n < (int64_t)kIndexSamples ? (uint32_t)n : kIndexSamples) &&
                    (n == 0 || (keys[0] == h.kmin && keys[n - 1] == h.kmax));
    IndexView v;
    index_layout((char *)index, h.n_leaves, h.nparams, h.root_segs, &v);
    // The fingerprint, shared out over the grid: the keys at the sampled
    // ranks must be the ones the index was trained on.  A difference is
    // reported (CGA_EMISMATCH); the ranks below stay exact for any sorted
    // array, because every window is verified.
    if (ok) {
        const uint32_t m = h.nsamples;
        for (uint64_t s = blockIdx.x + (uint64_t)threadIdx.x * gridDim.x; s < m;
             s += (uint64_t)gridDim.x * blockDim.x)
            if (keys[sample_rank((uint32_t)s, m, n)] != v.samp[s]) set_err(err, ERR_MISMATCH);
    }
    // every stride-th segment start, at most kLdsSegs of them, staged in LDS
    const uint32_t R = ok ? h.root_segs : 0;
    const uint32_t stride = R > kLdsSegs ? (R + kLdsSegs - 1) / kLdsSegs : 1;
    const uint32_t nrx = (R + stride - 1) / stride;
    for (uint32_t i = threadIdx.x; i < nrx; i += blockDim.x) s_rx[i] = v.rx[(size_t)i * stride];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq) return;
    if (!ok) {
        set_err(err, ERR_MISMATCH);
        rank[t] = 0;
        if (found) found[t] = 0;
        return;
    }
    const uint64_t x = q[t];
    int64_t r = 0;
    bool fell = false;
    if (n > 0) {
        const uint32_t j = route(h, v, s_rx, stride, nrx, x);
        const LeafHead lh = v.head(j);
        int64_t f0, f1;
        const int64_t p = leaf_predict(lh, v.params(j), h.leaf_kind, x, n, &f0, &f1);
        int64_t lo = p + lh.err_lo, hi = p + lh.err_hi;
        lo = lo < f0 ? f0 : (lo > f1 ? f1 : lo);
        hi = hi < lo ? lo : (hi > f1 ? f1 : hi);
        // The window [lo, hi] holds the answer iff keys[lo - 1] < x <=
        // keys[hi] (keys[-1] = -inf, keys[n] = +inf).  Both checks ride on
        // the search: the lower bound over [lo - 1, hi + 1) lands on lo - 1
        // exactly when keys[lo - 1] >= x and on hi + 1 exactly when
        // keys[hi] < x; anything between is the global lower bound.
        const int64_t sl = lo > 0 ? lo - 1 : 0, sh = hi < n ? hi + 1 : n;
        r = lb_range(keys, sl, sh, x);
        if ((lo > 0 && r == lo - 1) || (hi < n && r == hi + 1)) {
            r = lb_range(keys, (int64_t)0, n, x);
            fell = true;
        }
    }
    rank[t] = r;
    if (found) found[t] = (uint8_t)(r < n && keys[r] == x);
    if (fallbacks) {
        const uint64_t m = ballot64(fell);
        if (m && lane_id() == __ffsll((long long)__ballot(1)) - 1)
            atomicAdd(fallbacks, (unsigned long long)__popcll(m));
    }
}

__global__ void k_index_stats(const char *index, int32_t *width, int64_t *count) {
    const IndexHeader &h = *(const IndexHeader *)index;
    IndexView v;
    index_layout((char *)index, h.n_leaves, h.nparams, h.root_segs, &v);
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < h.n_leaves;
         j += gridDim.x * blockDim.x) {
        const LeafHead &lh = v.head(j);
        if (width) width[j] = lh.count ? lh.err_hi - lh.err_lo + 1 : 0;
        if (count) count[j] = lh.count;
    }
}

// The gradient the training uses, over n ascending samples in chunks of
// kMlpBatch (each chunk's units are active on a run of it).  Samples that do
// not ascend make every output NaN.
__global__ __launch_bounds__(kLeafBlock) void k_mlp_loss_grad(const float *params, const float *x,
                                                              const float *t, int64_t n,
                                                              double *grad, double *loss) {
    __shared__ float s_x[kMlpSlots], s_t[kMlpSlots], s_l0[kMlpSlots], s_l1[kMlpSlots], s_p[kMlpPad];
    __shared__ double s_e0[64], s_e1[64];
    const int tid = threadIdx.x;
    s_p[tid] = tid < kMlpParams ? params[tid] : 0.0f;
    bool bad = false;
    double g = 0.0, l2 = 0.0;
    for (int64_t base = 0; base < n; base += kMlpBatch) {
        const int m = n - base < kMlpBatch ? (int)(n - base) : kMlpBatch;
        __syncthreads();  // the previous chunk is consumed
        for (int i = tid; i < m; i += kLeafBlock) {
            s_x[lds_pad(i)] = x[base + i];
            s_t[lds_pad(i)] = t[base + i];
            bad |= base + i > 0 && !(x[base + i] >= x[base + i - 1]);
        }
        __syncthreads();
        double l;
        g += mlp_grad(s_p, s_x, s_t, m, s_l0, s_l1, s_e0, s_e1, tid, &l);
        l2 += l;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l2 += __shfl_xor(l2, o, 64);
    const double nan = __builtin_nan("");
    const bool any_bad = __ballot(bad) != 0;
    const double dn = n ? (double)n : 1.0;
    if (tid < kMlpParams) grad[tid] = any_bad ? nan : g / dn;
    if (tid == 0 && loss) *loss = any_bad ? nan : l2 / dn;
}

constexpr int kRootBlocks = 512;

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_index_bytes(const cga_index_params *p) {
    if (!p || p->n_leaves < 1 || p->n_leaves > kMaxLeaves || p->leaf_kind > 1) return 0;
    if (p->root_segments > 65536) return 0;
    return index_layout(nullptr, p->n_leaves, p->leaf_kind ? kMlpParams : 2, p->root_segments,
                        nullptr);
}

size_t cga_index_train_workspace_bytes(const cga_index_params *p, int64_t n) {
    if (!p || n < 0 || p->n_leaves < 1 || p->n_leaves > kMaxLeaves) return 0;
    return kControlBytes + idx_align((size_t)kRootBlocks * 4 * sizeof(double)) +
           idx_align(((size_t)p->n_leaves + 1) * sizeof(int64_t)) +
           idx_align(((size_t)p->n_leaves + kFirstTile) / kFirstTile * sizeof(int64_t));
}

int cga_index_train(const uint64_t *d_keys, int64_t n, const cga_index_params *p, void *d_index,
                    size_t index_bytes, void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!p || n < 0 || !d_index || !d_ws) return CGA_EINVAL;
    if (n > 0 && !d_keys) return CGA_EINVAL;
    if (n >= ((int64_t)1 << 31) - 1) return CGA_EUNSUPPORTED;
    const size_t need = cga_index_bytes(p);
    if (need == 0 || !(p->lr >= 0.0f)) return CGA_EINVAL;
    if (index_bytes < need) return CGA_EINVAL;
    if (ws_bytes < cga_index_train_workspace_bytes(p, n)) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Control *ctl = (Control *)d_ws;
    double *partial = (double *)((char *)d_ws + kControlBytes);
    int64_t *first =
        (int64_t *)((char *)d_ws + kControlBytes + idx_align((size_t)kRootBlocks * 4 * sizeof(double)));
    int64_t *tile_min = (int64_t *)((char *)first + idx_align(((size_t)p->n_leaves + 1) * sizeof(int64_t)));
    const uint32_t L = p->n_leaves, np = p->leaf_kind ? kMlpParams : 2;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    char *idx = (char *)d_index;
    IndexHeader *h = (IndexHeader *)idx;
    {
        CGA_PROF("index_root", s);
        k_index_header<<<1, 64, 0, s>>>(d_keys, n, L, p->leaf_kind, np, p->root_segments, h);
        if (n > 0) {
            k_index_samples<<<kIndexSamples / 256, 256, 0, s>>>(d_keys, n, idx);
            k_root_partial<<<kRootBlocks, 256, 0, s>>>(d_keys, n, h, partial);
            k_root_final<<<1, 256, 0, s>>>(partial, kRootBlocks, n, h);
            if (p->root_segments) {
                const unsigned rb = (p->root_segments + 255) / 256;
                k_root_knots<<<rb, 256, 0, s>>>(d_keys, n, idx);
            }
        }
    }
    int64_t blocks = (n + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    {
        CGA_PROF("index_bounds", s);
        const int64_t cnt = (int64_t)L + 1, tiles = (cnt + kFirstTile - 1) / kFirstTile;
        const int64_t fb = (cnt + 255) / 256 < 4096 ? (cnt + 255) / 256 : 4096;
        k_leaf_first_fill<<<(unsigned)fb, 256, 0, s>>>(first, cnt, n);
        if (n > 0) k_leaf_first_scatter<<<(unsigned)blocks, 256, 0, s>>>(d_keys, n, idx, first);
        k_leaf_first_tiles<<<(unsigned)tiles, kFirstBlock, 0, s>>>(first, cnt, tile_min);
        k_leaf_first_suffix<<<(unsigned)tiles, kFirstBlock, 0, s>>>(first, cnt, tile_min, tiles);
    }
    {
        CGA_PROF("index_fit", s);
        if (p->leaf_kind == 0)
            k_leaf_fit_linear<<<L, kLeafBlock, 0, s>>>(d_keys, idx, first);
        else
            k_leaf_fit_mlp<<<L, kLeafBlock, 0, s>>>(d_keys, idx, first, p->epochs, p->lr);
    }
    if (n > 0) {
        CGA_PROF("index_err", s);
        k_leaf_err<<<(unsigned)blocks, 256, 0, s>>>(d_keys, n, idx);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

size_t cga_index_lookup_workspace_bytes(void) { return kControlBytes; }

int cga_index_lookup(const void *d_index, const uint64_t *d_keys, int64_t n, const uint64_t *d_q,
                     int64_t nq, int64_t *d_rank, uint8_t *d_found, uint64_t *d_fallbacks,
                     void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!d_index || n < 0 || nq < 0 || !d_ws) return CGA_EINVAL;
    if ((n > 0 && !d_keys) || (nq > 0 && (!d_q || !d_rank))) return CGA_EINVAL;
    if (ws_bytes < kControlBytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Control *ctl = (Control *)d_ws;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (nq > 0) {
        CGA_PROF("index_lookup", s);
        k_index_lookup<<<(unsigned)((nq + kLookupBlock - 1) / kLookupBlock), kLookupBlock, 0, s>>>(
            (const char *)d_index, d_keys, n, d_q, nq, d_rank, d_found,
            (unsigned long long *)d_fallbacks, &ctl->err);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

int cga_index_stats(const void *d_index, int32_t *d_width, int64_t *d_count, cga_stream stream) {
    if (!d_index) return CGA_EINVAL;
    k_index_stats<<<256, 256, 0, (hipStream_t)stream>>>((const char *)d_index, d_width, d_count);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

int cga_mlp_loss_grad(const float *d_params, const float *d_x, const float *d_t, int64_t n,
                      double *d_grad, double *d_loss, cga_stream stream) {
    if (!d_params || !d_grad || n < 0 || (n > 0 && (!d_x || !d_t))) return CGA_EINVAL;
    k_mlp_loss_grad<<<1, kLeafBlock, 0, (hipStream_t)stream>>>(d_params, d_x, d_t, n, d_grad,
                                                               d_loss);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
