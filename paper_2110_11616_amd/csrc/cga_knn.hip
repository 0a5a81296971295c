// k-nearest-neighbour search, Eq. (7)-(8) generalised to k, over a sorted
// unique MORTON key array, and plain binary-search point lookup.
//
// Morton keys make every octree cell a contiguous key range: cell (prefix,
// L) holds exactly the keys in [prefix << 3L, (prefix + 1) << 3L).  One thread
// answers one query:
//  1. Binary-search the query's own key, then gallop outward from that
//     position to get the key range of every cell that contains the query,
//     from the voxel (level 0) up to the root -- O(log n) probes in total, all
//     near one place in the array.
//  2. Scan the query's voxel, then for each containing cell from the bottom
//     up visit its other seven children nearest-first (the child on the
//     query's side first, then those across one, two, three faces).  Inside a
//     visited child the same nearest-first order recurses without a stack:
//     the order of a child among its siblings follows from its own index bits
//     and the query's, and the key range of each open ancestor is kept per
//     level in LDS.  A cell whose nearest point is farther than the current
//     k-th distance is skipped (strictly farther, so ties survive); a cell
//     with at most a threshold number of keys is scanned exactly.
//  3. Stop climbing as soon as every point outside the finished cell is
//     farther than the current k-th distance.
// Candidates are kept in registers ordered by (squared distance, key); key
// order is array order.
#include <cstdlib>

#include "cga_common.h"
#include "cga_sort.h"

namespace cga {

constexpr int kKnnBlock = 256;
constexpr int kScanDefault = 16;  // scan a cell outright when it holds at most this many keys
// Queries are answered in the order of the top kOrderBits of their own keys,
// so that the lanes of a wave walk neighbouring cells (sorted by index with
// the onesweep sort when there are at least kOrderMin queries).
constexpr int kOrderBits = 24;
constexpr int64_t kOrderMin = 4096;

struct Cand {
    uint64_t d;
    int32_t i;
};

__device__ __forceinline__ bool cand_lt(uint64_t d, int32_t i, const Cand &c) {
    return d < c.d || (d == c.d && i < c.i);
}

// Ascending list of KT candidates, the last k of which are the answer; the
// first KT - k slots hold (0, -1) sentinels that no real candidate precedes.
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

// First index in [lo, hi) whose key is >= t (hi if none).
template <typename K>
__device__ __forceinline__ int32_t lower_bound_in(const K *keys, int32_t lo, int32_t hi, uint64_t t) {
    while (lo < hi) {
        int32_t mid = (int32_t)(((uint32_t)lo + (uint32_t)hi) >> 1);
        if ((uint64_t)keys[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First index >= lo whose key is >= t, given every key before lo is < t.
template <typename K>
__device__ __forceinline__ int64_t gallop_up(const K *keys, int64_t n, int64_t lo, uint64_t t) {
    if (lo >= n || (uint64_t)keys[lo] >= t) return lo;
    int64_t bad = lo, step = 1, good = n;  // keys[bad] < t, keys[good] >= t (or good == n)
    for (;;) {
        int64_t nx = bad + step;
        if (nx >= n) break;
        if ((uint64_t)keys[nx] >= t) {
            good = nx;
            break;
        }
        bad = nx;
        step <<= 1;
    }
    int64_t a = bad + 1, b = good;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if ((uint64_t)keys[mid] < t) a = mid + 1;
        else b = mid;
    }
    return a;
}

// First index whose key is >= t, given every key from hi on is >= t.
template <typename K>
__device__ __forceinline__ int64_t gallop_down(const K *keys, int64_t hi, uint64_t t) {
    if (hi <= 0 || (uint64_t)keys[hi - 1] < t) return hi;
    int64_t good = hi - 1, step = 1, bad = -1;  // keys[good] >= t, keys[bad] < t (or -1)
    for (;;) {
        int64_t nx = good - step;
        if (nx < 0) break;
        if ((uint64_t)keys[nx] < t) {
            bad = nx;
            break;
        }
        good = nx;
        step <<= 1;
    }
    int64_t a = bad + 1, b = good;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if ((uint64_t)keys[mid] < t) a = mid + 1;
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

// Visiting order of the 8 children: by the number of axes on which the child
// lies across from the query (0, 1, 1, 1, 2, 2, 2, 3).  Self-inverse.
__device__ __forceinline__ uint32_t near_order(uint32_t s) { return s == 3 ? 4u : (s == 4 ? 3u : s); }

template <typename K, int KT>
__global__ __launch_bounds__(kKnnBlock) void k_knn(const K *__restrict__ keys, int64_t n_host,
                                                   const int64_t *d_n, const float *__restrict__ q,
                                                   int64_t nq, float o0, float o1, float o2,
                                                   float scale, uint32_t depth, int k,
                                                   int scan_max,
                                                   const uint64_t *__restrict__ order,
                                                   int64_t *__restrict__ idx_out,
                                                   uint64_t *__restrict__ d2_out, uint32_t *err) {
    // key range [lo, hi) of the open cell at each level, one column per thread
    extern __shared__ int32_t s_rng[];
    int32_t *LO = s_rng + threadIdx.x;
    int32_t *HI = s_rng + (depth + 1) * kKnnBlock + threadIdx.x;
#define RLO(l) LO[(l) * kKnnBlock]
#define RHI(l) HI[(l) * kKnnBlock]

    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq) return;
    const int64_t j = order ? (int64_t)(order[t] >> kOrderBits) : t;
    const int64_t n = dev_count(n_host, d_n);
    const float o[3] = {o0, o1, o2};
    Vox qv;
    if (!quantize3(q[3 * j], q[3 * j + 1], q[3 * j + 2], o, scale, depth, qv)) {
        if (!order) set_err(err, ERR_NONFINITE);  // else reported by the ordering pass
        for (int s = 0; s < k; ++s) {
            idx_out[j * k + s] = -1;
            d2_out[j * k + s] = ~0ull;
        }
        return;
    }

    Cand e[KT];
#pragma unroll
    for (int s = 0; s < KT; ++s) e[s] = s < KT - k ? Cand{0, -1} : Cand{~0ull, 0x7FFFFFFF};

    const uint64_t qkey = enc3(qv.x, qv.y, qv.z, depth, false);
    // query's octant bits below each level: child index of the cell holding q
    auto qo = [&](int l) -> uint32_t {
        return (((qv.x >> l) & 1u) << 2) | (((qv.y >> l) & 1u) << 1) | ((qv.z >> l) & 1u);
    };

    // 1. range of the query's own voxel; the ranges of larger cells that
    // contain the query are galloped out from it as the climb needs them
    int64_t glo, ghi;
    {
        const int64_t p = lower_bound_dev(keys, n, (K)qkey);
        glo = gallop_down(keys, p, qkey);
        ghi = gallop_up(keys, n, p, qkey + 1);
        RLO(0) = (int32_t)glo;
        RHI(0) = (int32_t)ghi;
    }

    auto scan = [&](int32_t lo, int32_t hi) {
        for (int32_t i = lo; i < hi; ++i) {
            Vox v = dec3(keys[i], depth, false);
            cand_insert<KT>(e, sq_dist(v, qv.x, qv.y, qv.z), i);
        }
    };
    auto pruned = [&](uint64_t prefix, int l) {
        const uint32_t bx = compact3(prefix >> 2) << l, by = compact3(prefix >> 1) << l,
                       bz = compact3(prefix) << l;
        const uint32_t ext = (1u << l) - 1;
        const uint64_t gx = axis_gap(qv.x, bx, bx + ext), gy = axis_gap(qv.y, by, by + ext),
                       gz = axis_gap(qv.z, bz, bz + ext);
        return gx * gx + gy * gy + gz * gz > e[KT - 1].d;
    };

    // 2. the query's voxel, then the other children of each containing cell
    scan(RLO(0), RHI(0));
    for (int lp = 1; lp <= (int)depth; ++lp) {
        // 3. every point outside the finished cell (level lp - 1) is at least
        // this far along some axis
        {
            const int lc = lp - 1;
            const uint32_t c[3] = {qv.x, qv.y, qv.z};
            uint64_t m = ~0ull;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t b = (c[a] >> lc) << lc;
                const uint64_t below = (uint64_t)(c[a] - b) + 1, above = (uint64_t)b + (1u << lc) - c[a];
                const bool has_below = b > 0, has_above = (uint64_t)b + (1u << lc) <= ((1ull << depth) - 1);
                if (has_below && below < m) m = below;
                if (has_above && above < m) m = above;
            }
            if (m == ~0ull || (e[KT - 1].d != ~0ull && m * m > e[KT - 1].d)) break;
        }
        {
            const uint64_t cs = (qkey >> (3 * lp)) << (3 * lp);
            const uint64_t ce = cs + (1ull << (3 * lp));
            glo = gallop_down(keys, glo, cs);
            ghi = gallop_up(keys, n, ghi, ce);
            RLO(lp) = (int32_t)glo;
            RHI(lp) = (int32_t)ghi;
        }
        if (RHI(lp) - RLO(lp) == RHI(lp - 1) - RLO(lp - 1)) continue;  // no other keys here
        const uint64_t parent = qkey >> (3 * lp);
        const uint32_t qc = qo(lp - 1);
        for (uint32_t sidx = 1; sidx < 8; ++sidx) {
            // walk the subtree of sibling `sidx` (level lr = lp - 1) nearest-first
            const int lr = lp - 1;
            uint64_t prefix = (parent << 3) | (near_order(sidx) ^ qc);
            int l = lr;
            for (;;) {
                if (!pruned(prefix, l)) {
                    const int sh = 3 * l;
                    const uint64_t cs = prefix << sh, ce = (prefix + 1) << sh;
                    const int32_t lo = lower_bound_in(keys, RLO(l + 1), RHI(l + 1), cs);
                    const int32_t hi = lower_bound_in(keys, lo, RHI(l + 1), ce);
                    if (hi > lo) {
                        if (l == 0 || hi - lo <= scan_max) {
                            scan(lo, hi);
                        } else {
                            RLO(l) = lo;
                            RHI(l) = hi;
                            prefix = (prefix << 3) | qo(l - 1);  // first child: the query's side
                            --l;
                            continue;
                        }
                    }
                }
                // next cell: following sibling in nearest-first order, climbing
                // out of finished parents, until the subtree root is done
                bool done = false;
                for (;;) {
                    if (l == lr) {
                        done = true;
                        break;
                    }
                    const uint32_t so = near_order((uint32_t)(prefix & 7) ^ qo(l));
                    if (so < 7) {
                        prefix = (prefix & ~7ull) | (near_order(so + 1) ^ qo(l));
                        break;
                    }
                    prefix >>= 3;
                    ++l;
                }
                if (done) break;
            }
        }
    }
#undef RLO
#undef RHI

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


// ------------------------------------------------------------------------
// Team search: eight lanes answer one query together.
//
// A directory D over the top 21 key bits (cells at level T = depth - 7, or
// every voxel when depth <= 7) gives the key range of any cell at level >= T
// with two loads: D[c] = number of keys below cell c.  Round 0 splits the
// directory cell that holds the query among the lanes (lane t walks its
// t-th child in nearest-first order).  If the k-th distance found does not
// prove the answer lies inside that cell, later rounds cover the box of
// half-width r = floor(sqrt(bound)) around the query with the <= 2x2x2 cells
// of the smallest level whose edge spans it, one cell per lane.  All lanes
// prune with the best k-th distance any of them holds (one LDS word per
// team).  After each round the lanes' sorted lists are merged by a three-step
// butterfly of shuffles (bitonic min-merge), so every lane holds the team's
// list.  A round is exact when it starts from a known bound whose ball the
// box covers; otherwise the team restarts with the bound it now has (or a
// box twice as wide while fewer than k voxels were seen).
// ------------------------------------------------------------------------
constexpr int kTeam = 8;
constexpr int kTeamsPerBlock = kKnnBlock / kTeam;

__host__ __device__ inline int dir_level(uint32_t depth) { return depth > 7 ? (int)depth - 7 : 0; }
__host__ __device__ inline int64_t dir_cells(uint32_t depth) {
    return (int64_t)1 << (3 * ((int)depth - dir_level(depth)));
}

// D[c] for c in [0, NC]: one thread per cell.  Two lanes of each block first
// find the key range of the block's 256 consecutive cells; every thread then
// searches only inside it, so a thread needs a few probes, not log2(n).
template <typename K>
__global__ __launch_bounds__(256) void k_knn_dir(const K *__restrict__ keys, int64_t n_host,
                                                 const int64_t *d_n, int T, int64_t nc,
                                                 uint32_t *__restrict__ dir) {
    __shared__ int32_t s_lim[2];
    const int32_t n = (int32_t)dev_count(n_host, d_n);
    const int64_t b0 = (int64_t)blockIdx.x * 256;
    if (threadIdx.x < 2) {
        const int64_t c = b0 + (threadIdx.x == 0 ? 0 : 256);
        s_lim[threadIdx.x] = c > nc ? n : lower_bound_in(keys, 0, n, (uint64_t)c << (3 * T));
    }
    __syncthreads();
    const int64_t c = b0 + threadIdx.x;
    if (c > nc) return;
    dir[c] = (uint32_t)lower_bound_in(keys, s_lim[0], s_lim[1], (uint64_t)c << (3 * T));
}

__device__ __forceinline__ uint32_t isqrt64(uint64_t v) {
    uint64_t r = (uint64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (uint32_t)r;
}

// The team kernel keeps its candidate list as two register arrays (squared
// distance, key index) rather than an array of structs: whole-struct swaps
// would be lowered to memory copies and push the list out to scratch.
__device__ __forceinline__ bool cand_less2(uint64_t ad, int32_t ai, uint64_t bd, int32_t bi) {
    return ad < bd || (ad == bd && ai < bi);
}

// Insert into an ascending list of KT entries (the largest drops out).
template <int KT>
__device__ __forceinline__ void cand_insert2(uint64_t (&ed)[KT], int32_t (&ei)[KT], uint64_t d,
                                             int32_t i) {
    if (!cand_less2(d, i, ed[KT - 1], ei[KT - 1])) return;
    bool placed = false;
#pragma unroll
    for (int s = KT - 1; s > 0; --s) {
        const bool sh = !placed && cand_less2(d, i, ed[s - 1], ei[s - 1]);
        const uint64_t nd = sh ? ed[s - 1] : (placed ? ed[s] : d);
        const int32_t ni = sh ? ei[s - 1] : (placed ? ei[s] : i);
        placed = placed || !sh;
        ed[s] = nd;
        ei[s] = ni;
    }
    if (!placed) {
        ed[0] = d;
        ei[0] = i;
    }
}

// k-th smallest distance of a sorted list: the largest of its first k
// entries.  Written as a predicated maximum because a select chain on
// s == k - 1 is folded back into a variable index, which would put the list
// in scratch memory.
template <int KT>
__device__ __forceinline__ uint64_t kth_dist(const uint64_t (&ed)[KT], int k) {
    uint64_t d = ed[0];
#pragma unroll
    for (int s = 1; s < KT; ++s) {
        const uint64_t v = s < k ? ed[s] : 0;
        d = v > d ? v : d;
    }
    return d;
}

// Merge the team's sorted lists (no sentinels here: each lane keeps its KT
// best, real or empty): after the three exchange steps every lane holds the
// KT smallest of the union.
template <int KT>
__device__ __forceinline__ void team_merge(uint64_t (&ed)[KT], int32_t (&ei)[KT]) {
#pragma unroll
    for (int step = 1; step < kTeam; step <<= 1) {
        uint64_t pd[KT];
        int32_t pi[KT];
#pragma unroll
        for (int s = 0; s < KT; ++s) {
            const uint32_t lo = __shfl_xor((uint32_t)ed[s], step, 64);
            const uint32_t hi = __shfl_xor((uint32_t)(ed[s] >> 32), step, 64);
            pd[s] = ((uint64_t)hi << 32) | lo;
            pi[s] = __shfl_xor(ei[s], step, 64);
        }
        // elementwise min against the reversed partner: a bitonic sequence
        // holding the KT smallest, then a bitonic merge network
#pragma unroll
        for (int s = 0; s < KT; ++s) {
            const uint64_t bd = pd[KT - 1 - s];
            const int32_t bi = pi[KT - 1 - s];
            const bool t = cand_less2(bd, bi, ed[s], ei[s]);
            ed[s] = t ? bd : ed[s];
            ei[s] = t ? bi : ei[s];
        }
#pragma unroll
        for (int j = KT / 2; j > 0; j >>= 1) {
#pragma unroll
            for (int s = 0; s < KT; ++s) {
                if ((s & j) == 0) {
                    const uint64_t ad = ed[s], bd = ed[s + j];
                    const int32_t ai = ei[s], bi = ei[s + j];
                    const bool t = cand_less2(bd, bi, ad, ai);
                    ed[s] = t ? bd : ad;
                    ei[s] = t ? bi : ai;
                    ed[s + j] = t ? ad : bd;
                    ei[s + j] = t ? ai : bi;
                }
            }
        }
    }
}

template <typename K, int KT>
__global__ __launch_bounds__(kKnnBlock) void k_knn_team(
    const K *__restrict__ keys, int64_t n_host, const int64_t *d_n, const uint32_t *__restrict__ dir,
    const float *__restrict__ q, int64_t nq, float o0, float o1, float o2, float scale,
    uint32_t depth, int k, int scan_max, int64_t *__restrict__ idx_out,
    uint64_t *__restrict__ d2_out, uint32_t *err) {
    extern __shared__ int32_t s_rng[];  // key ranges of open cells below the directory level
    __shared__ unsigned long long s_bound[kTeamsPerBlock];
    const int tid = threadIdx.x, team = tid / kTeam, tl = tid % kTeam;
    const int DT = dir_level(depth);
    int32_t *LO = s_rng + tid;
    int32_t *HI = s_rng + (DT > 0 ? DT : 1) * kKnnBlock + tid;
#define RLO(l) LO[(l) * kKnnBlock]
#define RHI(l) HI[(l) * kKnnBlock]
    if (tl == 0) s_bound[team] = ~0ull;
    __syncthreads();  // the only block-wide barrier; teams run independently after it
    const int64_t j = (int64_t)blockIdx.x * kTeamsPerBlock + team;
    if (j >= nq) return;

    const float o[3] = {o0, o1, o2};
    Vox qv;
    if (!quantize3(q[3 * j], q[3 * j + 1], q[3 * j + 2], o, scale, depth, qv)) {
        if (tl == 0) set_err(err, ERR_NONFINITE);
        for (int s = tl; s < k; s += kTeam) {
            idx_out[j * k + s] = -1;
            d2_out[j * k + s] = ~0ull;
        }
        return;
    }
    uint64_t ed[KT];
    int32_t ei[KT];
#pragma unroll
    for (int s = 0; s < KT; ++s) {
        ed[s] = ~0ull;
        ei[s] = 0x7FFFFFFF;
    }
    uint64_t kth = ~0ull;  // this lane's k-th distance

    const uint64_t qkey = enc3(qv.x, qv.y, qv.z, depth, false);
    auto qo = [&](int l) __attribute__((always_inline)) -> uint32_t {
        return (((qv.x >> l) & 1u) << 2) | (((qv.y >> l) & 1u) << 1) | ((qv.z >> l) & 1u);
    };
    int32_t sk_lo = 0, sk_hi = 0;  // key range already considered (skipped by scans)
    auto bound_now = [&]() __attribute__((always_inline)) -> uint64_t {
        const uint64_t b = s_bound[team];
        return kth < b ? kth : b;
    };
    auto scan = [&](int32_t lo, int32_t hi) __attribute__((always_inline)) {
        for (int32_t i = lo; i < hi; ++i) {
            if (i >= sk_lo && i < sk_hi) {
                i = sk_hi - 1;
                continue;
            }
            Vox v = dec3(keys[i], depth, false);
            cand_insert2<KT>(ed, ei, sq_dist(v, qv.x, qv.y, qv.z), i);
        }
        kth = kth_dist<KT>(ed, k);
        if (kth < s_bound[team]) atomicMin(&s_bound[team], (unsigned long long)kth);
    };
    auto pruned = [&](uint64_t prefix, int l) __attribute__((always_inline)) {
        const uint32_t bx = compact3(prefix >> 2) << l, by = compact3(prefix >> 1) << l,
                       bz = compact3(prefix) << l;
        const uint32_t ext = (1u << l) - 1;
        const uint64_t gx = axis_gap(qv.x, bx, bx + ext), gy = axis_gap(qv.y, by, by + ext),
                       gz = axis_gap(qv.z, bz, bz + ext);
        return gx * gx + gy * gy + gz * gz > bound_now();
    };
    // key range of cell (prefix, l): the directory at levels >= DT, else a
    // binary search in the parent's range
    auto cell_range = [&](uint64_t prefix, int l, int32_t &lo, int32_t &hi) __attribute__((always_inline)) {
        if (l >= DT) {
            const int sh = 3 * (l - DT);
            lo = (int32_t)dir[prefix << sh];
            hi = (int32_t)dir[(prefix + 1) << sh];
            return;
        }
        int32_t pl, ph;
        if (l + 1 >= DT) {
            const int sh = 3 * (l + 1 - DT);
            pl = (int32_t)dir[(prefix >> 3) << sh];
            ph = (int32_t)dir[((prefix >> 3) + 1) << sh];
        } else {
            pl = RLO(l + 1);
            ph = RHI(l + 1);
        }
        const int s3 = 3 * l;
        lo = lower_bound_in(keys, pl, ph, prefix << s3);
        hi = lower_bound_in(keys, lo, ph, (prefix + 1) << s3);
    };
    auto walk = [&](uint64_t prefix, int lr) __attribute__((always_inline)) {
        int l = lr;
        for (;;) {
            if (!pruned(prefix, l)) {
                int32_t lo, hi;
                cell_range(prefix, l, lo, hi);
                if (hi > lo && !(lo >= sk_lo && hi <= sk_hi)) {
                    if (l == 0 || hi - lo <= scan_max) {
                        scan(lo, hi);
                    } else {
                        if (l < DT) {
                            RLO(l) = lo;
                            RHI(l) = hi;
                        }
                        prefix = (prefix << 3) | qo(l - 1);  // first child: the query's side
                        --l;
                        continue;
                    }
                }
            }
            bool done = false;
            for (;;) {
                if (l == lr) {
                    done = true;
                    break;
                }
                const uint32_t so = near_order((uint32_t)(prefix & 7) ^ qo(l));
                if (so < 7) {
                    prefix = (prefix & ~7ull) | (near_order(so + 1) ^ qo(l));
                    break;
                }
                prefix >>= 3;
                ++l;
            }
            if (done) break;
        }
    };
    auto reset = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < KT; ++s) {
            ed[s] = ~0ull;
            ei[s] = 0x7FFFFFFF;
        }
        kth = ~0ull;
    };

    const uint32_t top = (1u << depth) - 1;
    // round 0: the directory cell holding the query, split over the lanes
    const uint64_t cq = qkey >> (3 * DT);
    const int32_t tlo = (int32_t)dir[cq], thi = (int32_t)dir[cq + 1];
    if (DT == 0) {
        if (tl == 0) scan(tlo, thi);
    } else {
        walk((cq << 3) | (near_order((uint32_t)tl) ^ qo(DT - 1)), DT - 1);
    }
    team_merge<KT>(ed, ei);
    kth = kth_dist<KT>(ed, k);
    uint64_t bound = kth;
    bool done;
    {
        // every voxel outside the directory cell is at least m away
        const uint32_t c[3] = {qv.x, qv.y, qv.z};
        uint64_t m = ~0ull;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t b = (c[a] >> DT) << DT;
            const uint64_t below = (uint64_t)(c[a] - b) + 1, above = (uint64_t)b + (1u << DT) - c[a];
            if (b > 0 && below < m) m = below;
            if ((uint64_t)b + (1u << DT) <= top && above < m) m = above;
        }
        done = m == ~0ull || (bound != ~0ull && m * m > bound);
    }
    sk_lo = tlo;
    sk_hi = thi;
    if (!done && tl != 0) reset();  // lane 0 carries the team's list into the next round
    uint32_t r = bound != ~0ull ? isqrt64(bound) : ((1u << DT) - 1) / 2;
    while (!done) {
        if (r > top) r = top;
        const bool exact = bound != ~0ull && isqrt64(bound) <= r;
        int ls = DT;
        while (ls < (int)depth && (1u << ls) < 2 * r + 1) ++ls;
        {
            const uint32_t c3[3] = {qv.x, qv.y, qv.z};
            uint32_t c[3];
            bool ok = true;
            const uint32_t m = near_order((uint32_t)tl);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t lo = c3[a] > r ? c3[a] - r : 0;
                const uint32_t hi = (uint64_t)c3[a] + r < top ? c3[a] + r : top;
                const uint32_t own = c3[a] >> ls, clo = lo >> ls, chi = hi >> ls;
                if ((m >> (2 - a)) & 1u) {
                    const uint32_t other = own == clo ? chi : clo;
                    ok = ok && other != own;
                    c[a] = other;
                } else {
                    c[a] = own;
                }
            }
            if (ok) walk((spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]), ls);
        }
        team_merge<KT>(ed, ei);
        kth = kth_dist<KT>(ed, k);
        if (exact || ls == (int)depth) break;
        // not exact yet: start over on the box the candidates now bound
        bound = kth;
        r = bound != ~0ull ? isqrt64(bound) : 2 * r + 1;
        reset();
        sk_lo = sk_hi = 0;
        if (tl == 0) s_bound[team] = bound;
    }
#undef RLO
#undef RHI
#pragma unroll
    for (int s = 0; s < KT; ++s) {
        if (s < k && (s % kTeam) == tl) {
            const bool real = ed[s] != ~0ull;
            idx_out[j * k + s] = real ? (int64_t)ei[s] : -1;
            d2_out[j * k + s] = real ? ed[s] : ~0ull;
        }
    }
}

// Query ordering key: query index above the top kOrderBits of its Morton key,
// with the digit histogram of the 8-bit sort passes over those bits.
__global__ __launch_bounds__(256) void k_knn_order(const float *__restrict__ q, int64_t nq, float o0,
                                                   float o1, float o2, float scale,
                                                   uint32_t depth, uint64_t *__restrict__ out,
                                                   uint32_t *hist, uint32_t *err) {
    constexpr int RB = 8, PASSES = kOrderBits / RB;
    __shared__ uint32_t s_h[PASSES << RB];
    __shared__ int s_bad;
    for (int i = threadIdx.x; i < (PASSES << RB); i += blockDim.x) s_h[i] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const float o[3] = {o0, o1, o2};
    const int drop = 3 * (int)depth > kOrderBits ? 3 * (int)depth - kOrderBits : 0;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x) {
        Vox v;
        bad |= !quantize3(q[3 * i], q[3 * i + 1], q[3 * i + 2], o, scale, depth, v);
        const uint64_t top = enc3(v.x, v.y, v.z, depth, false) >> drop;
        const uint64_t packed = ((uint64_t)i << kOrderBits) | top;
        out[i] = packed;
        hist_add<RB>(s_h, packed, PASSES);
    }
    if (bad) s_bad = 1;
    __syncthreads();
    hist_flush<RB>(s_h, hist, PASSES);
    if (threadIdx.x == 0 && s_bad) set_err(err, ERR_NONFINITE);
}

// Launch knobs (never change results): CGA_KNN_SCAN = scan threshold,
// CGA_KNN_ORDER = 1 to answer queries in the order of their Morton keys
// (measured slower here: it gathers the costliest queries into the same waves).
struct KnnKnobs {
    int scan = kScanDefault;
    bool order = false;
    bool team = true;
};
static KnnKnobs knn_knobs() {
    KnnKnobs k;
    if (const char *e = getenv("CGA_KNN_SCAN")) {
        int v = atoi(e);
        if (v >= 1 && v <= 4096) k.scan = v;
    }
    if (const char *e = getenv("CGA_KNN_ORDER")) k.order = atoi(e) != 0;
    if (const char *e = getenv("CGA_KNN_TEAM")) k.team = atoi(e) != 0;
    return k;
}

struct KnnLayout {
    Control *ctl;
    uint32_t *dir;
    SortWs sort;
    uint64_t *a, *b;
    size_t bytes;
};

static KnnLayout knn_layout(void *ws, int64_t nq, uint32_t depth) {
    KnnLayout L;
    Carve c(ws);
    L.ctl = c.take<Control>(1);
    L.dir = c.take<uint32_t>((size_t)dir_cells(depth) + 1);
    L.a = L.b = nullptr;
    if (nq >= kOrderMin && knn_knobs().order) {
        SortCfg cfg;
        cfg.radix_bits = 8;
        cfg.items = 16;
        sort_carve(c, L.sort, nq, kOrderBits, cfg);
        L.a = c.take<uint64_t>((size_t)nq);
        L.b = c.take<uint64_t>((size_t)nq);
    }
    L.bytes = c.size();
    return L;
}

template <typename K, int KT>
static void knn_launch(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                       const float *q, int64_t nq, int k, const uint64_t *order, int64_t *idx,
                       uint64_t *d2, uint32_t *err, const uint32_t *dir, hipStream_t s) {
    CGA_PROF("knn", s);
    if (dir) {
        const int dt = dir_level(g->depth);
        const size_t lds = (size_t)(dt > 0 ? dt : 1) * kKnnBlock * 2 * sizeof(int32_t);
        k_knn_team<K, KT><<<(unsigned)((nq + kTeamsPerBlock - 1) / kTeamsPerBlock), kKnnBlock, lds, s>>>(
            keys, n, d_n, dir, q, nq, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth,
            k, knn_knobs().scan, idx, d2, err);
        return;
    }
    const size_t lds = (size_t)(g->depth + 1) * kKnnBlock * 2 * sizeof(int32_t);
    k_knn<K, KT><<<(unsigned)((nq + kKnnBlock - 1) / kKnnBlock), kKnnBlock, lds, s>>>(
        keys, n, d_n, q, nq, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth, k,
        knn_knobs().scan, order, idx, d2, err);
}

template <typename K>
static void knn_dispatch(const cga_grid *g, const K *keys, int64_t n, const int64_t *d_n,
                         const float *q, int64_t nq, int k, const uint64_t *order, int64_t *idx,
                         uint64_t *d2, uint32_t *err, uint32_t *dir, hipStream_t s) {
    if (dir) {
        const int dt = dir_level(g->depth);
        const int64_t nc = dir_cells(g->depth);
        CGA_PROF("knn_dir", s);
        k_knn_dir<K><<<(unsigned)((nc + 1 + 255) / 256), 256, 0, s>>>(keys, n, d_n, dt, nc, dir);
    }
    if (k <= 1) knn_launch<K, 1>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
    else if (k <= 2) knn_launch<K, 2>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
    else if (k <= 4) knn_launch<K, 4>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
    else if (k <= 8) knn_launch<K, 8>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
    else if (k <= 16) knn_launch<K, 16>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
    else knn_launch<K, 32>(g, keys, n, d_n, q, nq, k, order, idx, d2, err, dir, s);
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
    return knn_layout(nullptr, nq, g->depth).bytes;
}

int cga_knn(const cga_grid *g, const void *d_keys, int64_t n, const int64_t *d_n, const float *d_q,
            int64_t nq, int k, int64_t *d_idx, uint64_t *d_d2, void *d_ws, size_t ws_bytes,
            cga_stream stream) {
    if (!grid_valid(g) || n < 0 || n > INT32_MAX || nq < 0 || k < 1 || k > 32 || !d_ws)
        return CGA_EINVAL;
    if (nq > 0 && (!d_q || !d_idx || !d_d2)) return CGA_EINVAL;
    if (n > 0 && !d_keys) return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_MORTON) return CGA_EUNSUPPORTED;
    if (n >= ((int64_t)1 << 31) - 1) return CGA_EUNSUPPORTED;
    if (nq >= ((int64_t)1 << (64 - kOrderBits))) return CGA_EUNSUPPORTED;
    KnnLayout L = knn_layout(d_ws, nq, g->depth);
    if (ws_bytes < L.bytes) return CGA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Control *ctl = L.ctl;
    const bool ordered = L.a != nullptr;
    CGA_TRY(launch_begin(ctl, ordered ? L.sort.hist : nullptr, ordered ? sort_zero_bytes(L.sort) : 0,
                         nullptr, 0, nullptr, s));
    if (nq > 0) {
        const uint64_t *order = nullptr;
        if (ordered) {
            int64_t blocks = (nq + 256 * 8 - 1) / (256 * 8);
            blocks = blocks > 1024 ? 1024 : blocks;
            {
                CGA_PROF("knn_order", s);
                k_knn_order<<<(unsigned)blocks, 256, 0, s>>>(d_q, nq, g->origin[0], g->origin[1],
                                                              g->origin[2], g->scale, g->depth, L.a,
                                                              L.sort.hist, &ctl->err);
            }
            // 3 passes: a -> b -> a -> b
            sort_launch<uint64_t>(L.sort, L.a, L.b, L.a, L.b, nq, nullptr, true, ctl->tile_ctr, s);
            order = L.b;
        }
        uint32_t *dir = knn_knobs().team ? L.dir : nullptr;
        if (wide_keys(g->depth))
            knn_dispatch<uint64_t>(g, (const uint64_t *)d_keys, n, d_n, d_q, nq, k, order, d_idx,
                                   d_d2, &ctl->err, dir, s);
        else
            knn_dispatch<uint32_t>(g, (const uint32_t *)d_keys, n, d_n, d_q, nq, k, order, d_idx,
                                   d_d2, &ctl->err, dir, s);
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
    CGA_PROF("binary_lookup", s);
    k_binary_lookup<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(d_keys, n, d_n, d_q, nq, d_rank,
                                                                d_found);
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
