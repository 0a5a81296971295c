/*
 * CGA oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what the CGA hot path
 * computes, written from "Compressed Geometric Arrays for Point Cloud
 * Processing" (Roodaki, Nazm Bojnordi).  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg load this library; the product path never
 * does.  It shares no code, header, table or constant with the HIP library.
 *
 * Readings of the paper that the oracle fixes (all listed in the design notes):
 *  - Grid: voxel = clamp(floor(fl32(fl32(p - o) * s)), 0, 2^d - 1) per axis,
 *    round-to-nearest subtract then multiply, never fused; a non-finite
 *    coordinate is an error.  (The paper's data is already integer voxels,
 *    Table II; its bounding box encloses all points, Section II-E.)
 *  - A CGA is a *set* of voxels (duplicates collapse, with a multiplicity),
 *    stored in ascending (x, y, z) order, Section V.
 *  - Keys: LINEAR = x<<2d | y<<d | z (the paper's array order); MORTON puts
 *    bit b of x, y, z at key bits 3b+2, 3b+1, 3b.  Both are written here as
 *    per-bit loops.
 *  - k-NN: the k voxels smallest in (squared distance, key), Eq. (7)-(8),
 *    with the query quantized by the same grid rule.
 *
 * Parity pins live in tests/ (closed forms, library routes, Table II, brute
 * force, finite differences).  Everything here is fp64 or exact integer
 * arithmetic, except the quantizer which is float32 by definition.
 */
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

using Voxel = std::array<uint32_t, 3>;  // (x, y, z); std::array compares lexicographically

constexpr int MODE_MORTON = 0;
constexpr int MODE_LINEAR = 1;

// Per-bit Morton interleave: bit b of x -> 3b+2, of y -> 3b+1, of z -> 3b.
uint64_t morton3(const Voxel &v, uint32_t depth) {
    uint64_t key = 0;
    for (uint32_t b = 0; b < depth; ++b) {
        key |= (uint64_t)((v[0] >> b) & 1u) << (3 * b + 2);
        key |= (uint64_t)((v[1] >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((v[2] >> b) & 1u) << (3 * b + 0);
    }
    return key;
}

Voxel demorton3(uint64_t key, uint32_t depth) {
    Voxel v{0, 0, 0};
    for (uint32_t b = 0; b < depth; ++b) {
        v[0] |= (uint32_t)((key >> (3 * b + 2)) & 1u) << b;
        v[1] |= (uint32_t)((key >> (3 * b + 1)) & 1u) << b;
        v[2] |= (uint32_t)((key >> (3 * b + 0)) & 1u) << b;
    }
    return v;
}

uint64_t linear3(const Voxel &v, uint32_t depth) {
    return ((uint64_t)v[0] << (2 * depth)) | ((uint64_t)v[1] << depth) | (uint64_t)v[2];
}

Voxel delinear3(uint64_t key, uint32_t depth) {
    const uint64_t m = (depth >= 64) ? ~0ull : ((1ull << depth) - 1);
    return Voxel{(uint32_t)((key >> (2 * depth)) & m), (uint32_t)((key >> depth) & m),
                 (uint32_t)(key & m)};
}

uint64_t encode(const Voxel &v, uint32_t depth, int mode) {
    return mode == MODE_LINEAR ? linear3(v, depth) : morton3(v, depth);
}

Voxel decode(uint64_t key, uint32_t depth, int mode) {
    return mode == MODE_LINEAR ? delinear3(key, depth) : demorton3(key, depth);
}

// 2D keys of the two coordinates left after an axis is dropped, kept in
// (x, y, z) order: u is the earlier axis, v the later one.
uint64_t key2(uint32_t u, uint32_t v, uint32_t depth, int mode) {
    if (mode == MODE_LINEAR) return ((uint64_t)u << depth) | (uint64_t)v;
    uint64_t key = 0;
    for (uint32_t b = 0; b < depth; ++b) {
        key |= (uint64_t)((u >> b) & 1u) << (2 * b + 1);
        key |= (uint64_t)((v >> b) & 1u) << (2 * b);
    }
    return key;
}

// Grid rule (reading of Section II-E's bounding box + Table II's integer data).
// Returns false for a non-finite coordinate.
bool quantize_point(const float *p, const float *origin, float scale, uint32_t depth, Voxel &v) {
    const float top = (float)((1u << depth) - 1u);  // exact for depth <= 24
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(p[a])) return false;
        volatile float t = p[a] - origin[a];  // fl32 subtract
        volatile float u = t * scale;         // fl32 multiply (separately rounded)
        float f = std::floor((float)u);
        if (!(f >= 0.0f)) f = 0.0f;  // also catches -inf
        if (f > top) f = top;
        v[a] = (uint32_t)f;
    }
    return true;
}

uint64_t sqdist(const Voxel &a, const Voxel &b) {
    uint64_t s = 0;
    for (int k = 0; k < 3; ++k) {
        int64_t d = (int64_t)a[k] - (int64_t)b[k];
        s += (uint64_t)(d * d);
    }
    return s;
}

}  // namespace

extern "C" {

/* Grid rule.  Returns 0, or -4 on a non-finite coordinate (vox then undefined). */
int or_quantize(const float *xyz, int64_t n, const float *origin, float scale, uint32_t depth,
                uint32_t *vox) {
    for (int64_t i = 0; i < n; ++i) {
        Voxel v;
        if (!quantize_point(xyz + 3 * i, origin, scale, depth, v)) return -4;
        vox[3 * i + 0] = v[0];
        vox[3 * i + 1] = v[1];
        vox[3 * i + 2] = v[2];
    }
    return 0;
}

void or_encode(const uint32_t *vox, int64_t n, uint32_t depth, int mode, uint64_t *keys) {
    for (int64_t i = 0; i < n; ++i)
        keys[i] = encode(Voxel{vox[3 * i], vox[3 * i + 1], vox[3 * i + 2]}, depth, mode);
}

void or_decode(const uint64_t *keys, int64_t n, uint32_t depth, int mode, uint32_t *vox) {
    for (int64_t i = 0; i < n; ++i) {
        Voxel v = decode(keys[i], depth, mode);
        vox[3 * i + 0] = v[0];
        vox[3 * i + 1] = v[1];
        vox[3 * i + 2] = v[2];
    }
}

void or_encode2(const uint32_t *u, const uint32_t *v, int64_t n, uint32_t depth, int mode,
                uint64_t *keys) {
    for (int64_t i = 0; i < n; ++i) keys[i] = key2(u[i], v[i], depth, mode);
}

/* CGA construction (Section V): the set of occupied voxels with the number of
 * input points in each, as keys in ascending key order.  Returns U, or -4 on a
 * non-finite coordinate. */
int64_t or_build(const float *xyz, int64_t n, const float *origin, float scale, uint32_t depth,
                 int mode, uint64_t *keys, uint32_t *counts) {
    std::map<Voxel, uint32_t> occ;
    for (int64_t i = 0; i < n; ++i) {
        Voxel v;
        if (!quantize_point(xyz + 3 * i, origin, scale, depth, v)) return -4;
        occ[v] += 1;
    }
    std::vector<std::pair<uint64_t, uint32_t>> kv;
    kv.reserve(occ.size());
    for (const auto &e : occ) kv.emplace_back(encode(e.first, depth, mode), e.second);
    std::sort(kv.begin(), kv.end());
    for (size_t j = 0; j < kv.size(); ++j) {
        keys[j] = kv[j].first;
        if (counts) counts[j] = kv[j].second;
    }
    return (int64_t)kv.size();
}

/* The paper's five coordinate arrays (Section V), from a voxel set given as
 * keys in either mode.  Readings: X_pointer is indexed by position in X_index
 * and counts distinct y per x; Y_pointer counts z per (x, y) pair; all three
 * levels ascending.  Output sizes: x_index nx, x_ptr nx+1, y_index nxy,
 * y_ptr nxy+1, z_index U (= n after dedupe). */
void or_arrays(const uint64_t *keys, int64_t n, uint32_t depth, int mode, uint32_t *x_index,
               int64_t *x_ptr, uint32_t *y_index, int64_t *y_ptr, uint32_t *z_index,
               int64_t *n_x, int64_t *n_xy, int64_t *n_z) {
    std::set<Voxel> vs;
    for (int64_t i = 0; i < n; ++i) vs.insert(decode(keys[i], depth, mode));
    int64_t nx = 0, nxy = 0, nz = 0;
    x_ptr[0] = 0;
    y_ptr[0] = 0;
    bool have = false;
    uint32_t cx = 0, cy = 0;
    for (const Voxel &v : vs) {
        if (!have || v[0] != cx) {  // new x: open a new X_index entry
            x_index[nx++] = v[0];
            x_ptr[nx] = x_ptr[nx - 1];
            cx = v[0];
            have = false;
        }
        if (!have || v[1] != cy) {  // new (x, y): one more distinct y for this x
            y_index[nxy++] = v[1];
            y_ptr[nxy] = y_ptr[nxy - 1];
            x_ptr[nx] += 1;
            cy = v[1];
            have = true;
        }
        z_index[nz++] = v[2];
        y_ptr[nxy] += 1;  // one more z for this (x, y)
    }
    *n_x = nx;
    *n_xy = nxy;
    *n_z = nz;
}

/* Merge, Eq. (1): S0 u S1 as sets of voxels, returned as ascending keys.
 * src (nullable): 1 = only in A, 2 = only in B, 3 = in both. */
int64_t or_merge(const uint64_t *a, int64_t na, const uint64_t *b, int64_t nb, uint32_t depth,
                 int mode, uint64_t *out, uint8_t *src) {
    std::set<Voxel> sa, sb;
    for (int64_t i = 0; i < na; ++i) sa.insert(decode(a[i], depth, mode));
    for (int64_t i = 0; i < nb; ++i) sb.insert(decode(b[i], depth, mode));
    std::vector<Voxel> u;
    std::set_union(sa.begin(), sa.end(), sb.begin(), sb.end(), std::back_inserter(u));
    std::vector<std::pair<uint64_t, uint8_t>> kv;
    kv.reserve(u.size());
    for (const Voxel &v : u)
        kv.emplace_back(encode(v, depth, mode),
                        (uint8_t)((sa.count(v) ? 1 : 0) | (sb.count(v) ? 2 : 0)));
    std::sort(kv.begin(), kv.end());
    for (size_t j = 0; j < kv.size(); ++j) {
        out[j] = kv[j].first;
        if (src) src[j] = kv[j].second;
    }
    return (int64_t)kv.size();
}

/* Orthogonal projection, Eq. (3) with m_x = m_y = 1, generalised to dropping
 * any one axis: the image of the voxel set as a set of 2D pixels, with the
 * number of voxels that fall on each pixel.  Ascending 2D keys. */
int64_t or_project(const uint64_t *keys, int64_t n, uint32_t depth, int mode, int drop_axis,
                   uint64_t *out, uint32_t *counts) {
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> img;
    std::set<Voxel> vs;
    for (int64_t i = 0; i < n; ++i) vs.insert(decode(keys[i], depth, mode));
    for (const Voxel &v : vs) {
        uint32_t u, w;
        if (drop_axis == 0) { u = v[1]; w = v[2]; }
        else if (drop_axis == 1) { u = v[0]; w = v[2]; }
        else { u = v[0]; w = v[1]; }
        img[{u, w}] += 1;
    }
    std::vector<std::pair<uint64_t, uint32_t>> kv;
    kv.reserve(img.size());
    for (const auto &e : img) kv.emplace_back(key2(e.first.first, e.first.second, depth, mode), e.second);
    std::sort(kv.begin(), kv.end());
    for (size_t j = 0; j < kv.size(); ++j) {
        out[j] = kv[j].first;
        if (counts) counts[j] = kv[j].second;
    }
    return (int64_t)kv.size();
}

/* k-NN by definition, Eq. (7)-(8): for each query, the k entries of the key
 * array smallest in (squared distance, key); key order equals array order, so
 * ties break toward the lower index.  Pads with (-1, UINT64_MAX).  Returns 0
 * or -4 for a non-finite query.  OpenMP over queries. */
int or_knn_brute(const uint64_t *keys, int64_t n, uint32_t depth, int mode, const float *q,
                 int64_t nq, const float *origin, float scale, int k, int64_t *idx, uint64_t *d2) {
    std::vector<Voxel> vs(n);
    for (int64_t i = 0; i < n; ++i) vs[i] = decode(keys[i], depth, mode);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t j = 0; j < nq; ++j) {
        Voxel qv;
        if (!quantize_point(q + 3 * j, origin, scale, depth, qv)) { bad = 1; continue; }
        std::vector<std::pair<uint64_t, int64_t>> all(n);
        for (int64_t i = 0; i < n; ++i) all[i] = {sqdist(qv, vs[i]), i};
        int64_t kk = std::min<int64_t>(k, n);
        std::partial_sort(all.begin(), all.begin() + kk, all.end());
        for (int t = 0; t < k; ++t) {
            idx[j * k + t] = t < kk ? all[t].second : -1;
            d2[j * k + t] = t < kk ? all[t].first : UINT64_MAX;
        }
    }
    return bad ? -4 : 0;
}

}  // extern "C"

/* ------------------------------------------------------------------------ */
/* kd-tree k-NN following Algorithm 1: descend to the leaf region of the     */
/* query, then unwind, testing each superior (ancestor) node's point and the  */
/* subtree on the other side of its splitting plane whenever a closer point   */
/* could lie there.  Ties are kept (a far side is visited when its plane      */
/* distance equals the current k-th distance) so the (distance, key) order    */
/* is exact.                                                                 */
/* ------------------------------------------------------------------------ */
namespace {

struct KdTree {
    std::vector<Voxel> pts;      // points permuted into tree order
    std::vector<int64_t> id;     // original index of each tree slot
    std::vector<uint8_t> axis;   // split axis of the node stored at each slot

    // Median split cycling x, y, z; the node point sits at the middle slot of
    // its range, its left subtree before it and its right subtree after it.
    void build(const std::vector<Voxel> &src) {
        const int64_t n = (int64_t)src.size();
        std::vector<int64_t> perm(n);
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        axis.assign(n, 0);
        split(src, perm, 0, n, 0);
        pts.resize(n);
        id.resize(n);
        for (int64_t i = 0; i < n; ++i) { pts[i] = src[perm[i]]; id[i] = perm[i]; }
    }

    void split(const std::vector<Voxel> &src, std::vector<int64_t> &perm, int64_t lo, int64_t hi,
               int level) {
        if (hi - lo <= 0) return;
        int64_t mid = lo + (hi - lo) / 2;
        int ax = level % 3;
        std::nth_element(perm.begin() + lo, perm.begin() + mid, perm.begin() + hi,
                         [&](int64_t a, int64_t b) {
                             if (src[a][ax] != src[b][ax]) return src[a][ax] < src[b][ax];
                             return a < b;
                         });
        axis[mid] = (uint8_t)ax;
        split(src, perm, lo, mid, level + 1);
        split(src, perm, mid + 1, hi, level + 1);
    }
};

struct TopK {
    int k;
    std::vector<std::pair<uint64_t, int64_t>> best;  // sorted ascending (d2, index)
    bool full() const { return (int)best.size() == k; }
    uint64_t worst() const { return best.back().first; }
    void offer(uint64_t d, int64_t i) {
        std::pair<uint64_t, int64_t> c{d, i};
        if (full() && !(c < best.back())) return;
        auto it = std::upper_bound(best.begin(), best.end(), c);
        best.insert(it, c);
        if ((int)best.size() > k) best.pop_back();
    }
};

void kd_search(const KdTree &t, int64_t lo, int64_t hi, const Voxel &q, TopK &top) {
    if (hi - lo <= 0) return;
    int64_t mid = lo + (hi - lo) / 2;
    int ax = t.axis[mid];
    const Voxel &p = t.pts[mid];
    bool go_left = q[ax] < p[ax];
    // descend toward the query's side first
    if (go_left) kd_search(t, lo, mid, q, top);
    else kd_search(t, mid + 1, hi, q, top);
    // unwinding: test the superior node's own point
    top.offer(sqdist(q, p), t.id[mid]);
    // test the other side if a point there could be as close as the current k-th
    int64_t dp = (int64_t)q[ax] - (int64_t)p[ax];
    uint64_t plane = (uint64_t)(dp * dp);
    if (!top.full() || plane <= top.worst()) {
        if (go_left) kd_search(t, mid + 1, hi, q, top);
        else kd_search(t, lo, mid, q, top);
    }
}

}  // namespace

extern "C" {

int or_knn_kdtree(const uint64_t *keys, int64_t n, uint32_t depth, int mode, const float *q,
                  int64_t nq, const float *origin, float scale, int k, int64_t *idx,
                  uint64_t *d2) {
    std::vector<Voxel> vs(n);
    for (int64_t i = 0; i < n; ++i) vs[i] = decode(keys[i], depth, mode);
    KdTree t;
    t.build(vs);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t j = 0; j < nq; ++j) {
        Voxel qv;
        if (!quantize_point(q + 3 * j, origin, scale, depth, qv)) { bad = 1; continue; }
        TopK top{k, {}};
        kd_search(t, 0, n, qv, top);
        for (int s = 0; s < k; ++s) {
            bool ok = s < (int)top.best.size();
            idx[j * k + s] = ok ? top.best[s].second : -1;
            d2[j * k + s] = ok ? top.best[s].first : UINT64_MAX;
        }
    }
    return bad ? -4 : 0;
}

/* The paper's own CGA nearest-neighbour search (Section V-C), 1-NN, on the
 * five coordinate arrays:
 *   1. look for a point equal to the query (three-level search, Section V-A);
 *   2. otherwise take the nearest x in X_index, then the nearest y among that
 *      x's Y_index entries, then the nearest z among that (x, y)'s Z_index
 *      entries; their distance is epsilon;
 *   3. every point whose x, y and z each lie within epsilon of the query's is
 *      a candidate; return the candidate with the smallest distance.
 * Readings: "within epsilon" is taken as <= so ties survive, and a tie in
 * distance goes to the smaller key of `mode` (the same order as the other
 * tiers).  Query voxels are given directly.  Writes the point's position in
 * Z_index order (= LINEAR key order) and its squared distance. */
void or_nn_cga(const uint32_t *x_index, int64_t nx, const int64_t *x_ptr, const uint32_t *y_index,
               const int64_t *y_ptr, const uint32_t *z_index, uint32_t depth, int mode,
               const uint32_t *qvox, int64_t nq, int64_t *pos_out, uint64_t *d2_out) {
    auto nearest = [](const uint32_t *arr, int64_t lo, int64_t hi, uint32_t v) {
        // index in [lo, hi) of the value closest to v (first of equals)
        int64_t bi = lo;
        uint64_t bd = UINT64_MAX;
        for (int64_t i = lo; i < hi; ++i) {
            int64_t d = (int64_t)arr[i] - (int64_t)v;
            uint64_t ad = (uint64_t)(d < 0 ? -d : d);
            if (ad < bd) { bd = ad; bi = i; }
        }
        return bi;
    };
    for (int64_t j = 0; j < nq; ++j) {
        Voxel q{qvox[3 * j], qvox[3 * j + 1], qvox[3 * j + 2]};
        if (nx == 0) { pos_out[j] = -1; d2_out[j] = UINT64_MAX; continue; }
        // steps 1-2: exact match falls out of the nearest-coordinate walk with distance 0
        int64_t xi = nearest(x_index, 0, nx, q[0]);
        int64_t yi = nearest(y_index, x_ptr[xi], x_ptr[xi + 1], q[1]);
        int64_t zi = nearest(z_index, y_ptr[yi], y_ptr[yi + 1], q[2]);
        Voxel f{x_index[xi], y_index[yi], z_index[zi]};
        uint64_t eps2 = sqdist(q, f);
        // step 3: candidate box |c - q| <= epsilon in every coordinate
        int64_t best = -1;
        uint64_t bd = UINT64_MAX, bkey = UINT64_MAX;
        for (int64_t a = 0; a < nx; ++a) {
            int64_t dx = (int64_t)x_index[a] - (int64_t)q[0];
            if ((uint64_t)(dx * dx) > eps2) continue;
            for (int64_t b = x_ptr[a]; b < x_ptr[a + 1]; ++b) {
                int64_t dy = (int64_t)y_index[b] - (int64_t)q[1];
                if ((uint64_t)(dy * dy) > eps2) continue;
                for (int64_t c = y_ptr[b]; c < y_ptr[b + 1]; ++c) {
                    int64_t dz = (int64_t)z_index[c] - (int64_t)q[2];
                    if ((uint64_t)(dz * dz) > eps2) continue;
                    Voxel v{x_index[a], y_index[b], z_index[c]};
                    uint64_t d = sqdist(q, v), key = encode(v, depth, mode);
                    if (d < bd || (d == bd && key < bkey)) { bd = d; bkey = key; best = c; }
                }
            }
        }
        pos_out[j] = best;
        d2_out[j] = bd;
    }
}

/* Point lookup on the five coordinate arrays, Section V-A: find the query's x
 * in X_index; its X_pointer entries bound that x's run of Y_index; find the
 * query's y in that run; its Y_pointer entries bound the (x, y) run of
 * Z_index; find the query's z there.  Reading: X_pointer is indexed by the
 * position of the x in X_index, not by the raw coordinate (the G-Arrays form
 * the text's formula keeps), and each "find" is a plain search of an
 * ascending run.  Writes the voxel's position in Z_index order (= the index
 * of its LINEAR key), or -1 when it is absent. */
void or_lookup_cga(const uint32_t *x_index, int64_t nx, const int64_t *x_ptr,
                   const uint32_t *y_index, const int64_t *y_ptr, const uint32_t *z_index,
                   const uint32_t *qvox, int64_t nq, int64_t *pos_out) {
    auto find = [](const uint32_t *arr, int64_t lo, int64_t hi, uint32_t v) -> int64_t {
        const uint32_t *p = std::lower_bound(arr + lo, arr + hi, v);
        return (p != arr + hi && *p == v) ? p - arr : -1;
    };
    for (int64_t j = 0; j < nq; ++j) {
        const uint32_t qx = qvox[3 * j], qy = qvox[3 * j + 1], qz = qvox[3 * j + 2];
        int64_t pos = -1;
        const int64_t a = find(x_index, 0, nx, qx);
        if (a >= 0) {
            const int64_t b = find(y_index, x_ptr[a], x_ptr[a + 1], qy);
            if (b >= 0) pos = find(z_index, y_ptr[b], y_ptr[b + 1], qz);
        }
        pos_out[j] = pos;
    }
}

/* Temporal prediction of one frame from a reference frame (Section V-D),
 * both given as CGAs (ascending unique keys of the grid's mode, one packed
 * 4 x 8-bit value per voxel):
 *   1. each frame's voxels are clustered by k-means with eight centres
 *      started at the corners of the frame's bounding box;
 *   2. cluster i of the predicted frame corresponds to cluster i of the
 *      reference (the same starting corner); its motion vector is the
 *      difference of the two centroids, rounded to whole voxels;
 *   3. every predicted voxel, moved back by its cluster's motion vector, is
 *      matched to the reference voxel of smallest SAD of the four channels
 *      among those within `window` voxels on every axis;
 *   4. the residual is the channel-wise difference predicted - matched.
 * Readings (the text fixes none of these): corner i has x = max when bit 2
 * of i is set (else min), y by bit 1, z by bit 0; distances to centres are
 * squared Euclidean in double precision, summed x, y, z without fused
 * multiply-add, ties to the lower cluster; a centre is the mean of its
 * voxels (exact integer sums, one division) and keeps its place when empty;
 * an iteration assigns every voxel, and the run stops at the first
 * assignment that repeats the previous one or after max_iter assignments
 * (so the final assignment is always nearest-centre for the final
 * centres); rounding is half away from zero; SAD ties go to the smaller
 * L1 coordinate distance, then to the smaller key; a voxel moved outside the
 * grid, or with no reference voxel in its window, has match -1, SAD
 * UINT32_MAX and its own channels as residual. */
static int kmeans8(const std::vector<Voxel> &pts, int max_iter, uint8_t *assign, double cent[8][3]) {
    const int64_t n = (int64_t)pts.size();
    uint32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            if (i == 0 || pts[i][a] < lo[a]) lo[a] = pts[i][a];
            if (i == 0 || pts[i][a] > hi[a]) hi[a] = pts[i][a];
        }
    for (int c = 0; c < 8; ++c)
        for (int a = 0; a < 3; ++a) cent[c][a] = (double)(((c >> (2 - a)) & 1) ? hi[a] : lo[a]);
    int it = 0;
    while (it < max_iter) {
        bool changed = false;
        for (int64_t i = 0; i < n; ++i) {
            int best = 0;
            double bd = 0.0;
            for (int c = 0; c < 8; ++c) {
                const double dx = (double)pts[i][0] - cent[c][0];
                const double dy = (double)pts[i][1] - cent[c][1];
                const double dz = (double)pts[i][2] - cent[c][2];
                const double d = dx * dx + dy * dy + dz * dz;
                if (c == 0 || d < bd) { bd = d; best = c; }
            }
            if (it == 0 || assign[i] != best) changed = true;
            assign[i] = (uint8_t)best;
        }
        ++it;
        if (!changed || it == max_iter) break;
        int64_t sum[8][3] = {}, cnt[8] = {};
        for (int64_t i = 0; i < n; ++i) {
            ++cnt[assign[i]];
            for (int a = 0; a < 3; ++a) sum[assign[i]][a] += pts[i][a];
        }
        for (int c = 0; c < 8; ++c)
            if (cnt[c] > 0)
                for (int a = 0; a < 3; ++a) cent[c][a] = (double)sum[c][a] / (double)cnt[c];
    }
    return it;
}

void or_temporal_predict(const uint64_t *ref_keys, const uint32_t *ref_vals, int64_t n_ref,
                         const uint64_t *pred_keys, const uint32_t *pred_vals, int64_t n_pred,
                         uint32_t depth, int mode, int window, int max_iter, uint8_t *ref_assign,
                         uint8_t *pred_assign, double *centroids, int32_t *mv, int32_t *iters,
                         int64_t *match, uint32_t *sad, int16_t *residual) {
    std::vector<Voxel> rv(n_ref), pv(n_pred);
    std::map<Voxel, int64_t> where;  // reference voxel -> index in its key array
    for (int64_t i = 0; i < n_ref; ++i) {
        rv[i] = decode(ref_keys[i], depth, mode);
        where[rv[i]] = i;
    }
    for (int64_t i = 0; i < n_pred; ++i) pv[i] = decode(pred_keys[i], depth, mode);
    double cr[8][3], cp[8][3];
    iters[0] = kmeans8(rv, max_iter, ref_assign, cr);
    iters[1] = kmeans8(pv, max_iter, pred_assign, cp);
    for (int c = 0; c < 8; ++c)
        for (int a = 0; a < 3; ++a) {
            centroids[c * 3 + a] = cr[c][a];
            centroids[24 + c * 3 + a] = cp[c][a];
            mv[c * 3 + a] = (int32_t)std::llround(cp[c][a] - cr[c][a]);
        }
    const int64_t top = (int64_t)1 << depth;
    auto chan = [](uint32_t v, int c) { return (int32_t)((v >> (8 * c)) & 0xFFu); };
    for (int64_t i = 0; i < n_pred; ++i) {
        int64_t r[3];
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            r[a] = (int64_t)pv[i][a] - mv[pred_assign[i] * 3 + a];
            inside = inside && r[a] >= 0 && r[a] < top;
        }
        int64_t best = -1;
        uint64_t bs = UINT64_MAX, bl = 0, bk = 0;
        if (inside) {
            for (int64_t dx = -window; dx <= window; ++dx)
                for (int64_t dy = -window; dy <= window; ++dy)
                    for (int64_t dz = -window; dz <= window; ++dz) {
                        const int64_t c[3] = {r[0] + dx, r[1] + dy, r[2] + dz};
                        if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= top || c[1] >= top || c[2] >= top)
                            continue;
                        const auto it = where.find(Voxel{(uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]});
                        if (it == where.end()) continue;
                        uint64_t sd = 0;
                        for (int ch = 0; ch < 4; ++ch)
                            sd += (uint64_t)std::abs(chan(pred_vals[i], ch) - chan(ref_vals[it->second], ch));
                        const uint64_t l1 = (uint64_t)(std::llabs(dx) + std::llabs(dy) + std::llabs(dz));
                        const uint64_t key = ref_keys[it->second];
                        if (best < 0 || sd < bs || (sd == bs && (l1 < bl || (l1 == bl && key < bk)))) {
                            best = it->second;
                            bs = sd;
                            bl = l1;
                            bk = key;
                        }
                    }
        }
        match[i] = best;
        sad[i] = best < 0 ? UINT32_MAX : (uint32_t)bs;
        for (int ch = 0; ch < 4; ++ch)
            residual[4 * i + ch] = (int16_t)(chan(pred_vals[i], ch) - (best < 0 ? 0 : chan(ref_vals[best], ch)));
    }
}

/* Point location / range start: rank = lower_bound(keys, q), found = key
 * present.  The exact contract every learned-index lookup must reproduce. */
void or_lower_bound(const uint64_t *keys, int64_t n, const uint64_t *q, int64_t nq, int64_t *rank,
                    uint8_t *found) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nq; ++j) {
        const uint64_t *p = std::lower_bound(keys, keys + n, q[j]);
        rank[j] = p - keys;
        if (found) found[j] = (uint8_t)(p != keys + n && *p == q[j]);
    }
}

/* Attribute payload: the Value array of Section V.  Each point carries four
 * 8-bit channels packed in a uint32 (channel c in bits 8c .. 8c + 7).  A
 * voxel's value is the channel-wise average of its points' values, as the
 * grid downsampling of Section III-B averages the colours of the points in
 * a box, each channel rounded half up: floor((2 sum + count) / (2 count)).
 * Outputs keys (ascending) and values; returns U, or -4 for a non-finite
 * coordinate. */
static uint32_t channel_average(const uint64_t sum[4], uint64_t count) {
    uint32_t v = 0;
    for (int c = 0; c < 4; ++c) {
        const uint64_t a = (2 * sum[c] + count) / (2 * count);
        v |= (uint32_t)a << (8 * c);
    }
    return v;
}

int64_t or_voxel_values(const float *xyz, int64_t n, const uint32_t *attr, const float *origin,
                        float scale, uint32_t depth, int mode, uint64_t *keys, uint32_t *values) {
    std::map<uint64_t, std::array<uint64_t, 5>> acc;  // channel sums, point count
    for (int64_t i = 0; i < n; ++i) {
        Voxel v;
        if (!quantize_point(xyz + 3 * i, origin, scale, depth, v)) return -4;
        auto &a = acc[encode(v, depth, mode)];
        for (int c = 0; c < 4; ++c) a[c] += (attr[i] >> (8 * c)) & 0xFFu;
        a[4] += 1;
    }
    int64_t u = 0;
    for (const auto &kv : acc) {
        keys[u] = kv.first;
        values[u] = channel_average(kv.second.data(), kv.second[4]);
        ++u;
    }
    return u;
}

/* Values of a merge, Eq. (1): a voxel of only one cloud keeps its value; a
 * voxel of both keeps the base cloud's (a's) value under policy 0, or takes
 * the channel-wise average of the two values (rounded half up) under policy
 * 1 -- the two choices Section II-A gives for overlapping points.  Returns
 * the union size. */
int64_t or_merge_values(const uint64_t *ka, const uint32_t *va, int64_t na, const uint64_t *kb,
                        const uint32_t *vb, int64_t nb, int policy, uint64_t *keys,
                        uint32_t *values) {
    std::map<uint64_t, uint32_t> m;
    for (int64_t i = 0; i < na; ++i) m[ka[i]] = va[i];
    for (int64_t i = 0; i < nb; ++i) {
        auto it = m.find(kb[i]);
        if (it == m.end()) {
            m[kb[i]] = vb[i];
        } else if (policy == 1) {
            uint64_t sum[4];
            for (int c = 0; c < 4; ++c)
                sum[c] = ((it->second >> (8 * c)) & 0xFFu) + ((vb[i] >> (8 * c)) & 0xFFu);
            it->second = channel_average(sum, 2);
        }
    }
    int64_t u = 0;
    for (const auto &kv : m) {
        keys[u] = kv.first;
        values[u] = kv.second;
        ++u;
    }
    return u;
}

/* Octree occupancy codes (Section II-E, point cloud compression: constructing
 * the octree, coding of the occupancy codes).  The octree of a MORTON key set
 * has, at level L, one occupied cell per distinct key >> 3L; a cell's 8-bit
 * code has bit o set when its child in octant o (child prefix = prefix * 8 +
 * o, o = x_bit << 2 | y_bit << 1 | z_bit) is occupied.  The codes are written
 * from the root (L = depth) down to L = 1, level by level, cells of a level in
 * key order.  counts[L] = occupied cells at level L (counts[0] = voxels).
 * Returns the number of codes. */
int64_t or_occupancy(const uint64_t *keys, int64_t n, uint32_t depth, uint8_t *occ,
                     int64_t *counts) {
    std::vector<std::set<uint64_t>> cells(depth + 1);
    for (int64_t i = 0; i < n; ++i)
        for (uint32_t L = 0; L <= depth; ++L) cells[L].insert(keys[i] >> (3 * L));
    for (uint32_t L = 0; L <= depth; ++L) counts[L] = (int64_t)cells[L].size();
    int64_t t = 0;
    for (int L = (int)depth; L >= 1; --L)
        for (uint64_t c : cells[L]) {
            uint8_t m = 0;
            for (uint32_t o = 0; o < 8; ++o)
                if (cells[L - 1].count(c * 8 + o)) m |= (uint8_t)(1u << o);
            occ[t++] = m;
        }
    return t;
}

/* 1-16-1 ReLU network f(x) = sum_h w2[h] relu(w1[h] x + b1[h]) + b2 and its
 * mean-squared-error loss L = (1/n) sum_i (f(x_i) - t_i)^2, with the analytic
 * gradient in fp64.  Parameter order: w1[16], b1[16], w2[16], b2.  Returns L.
 * kink (nullable) counts samples with a hidden pre-activation exactly 0. */
double or_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t n,
                        double *grad, int64_t *kink) {
    const double *w1 = p, *b1 = p + 16, *w2 = p + 32;
    const double b2 = p[48];
    double g[49];
    std::memset(g, 0, sizeof g);
    double loss = 0.0;
    int64_t kinks = 0;
    for (int64_t i = 0; i < n; ++i) {
        double z[16], h[16], f = b2;
        for (int j = 0; j < 16; ++j) {
            z[j] = w1[j] * x[i] + b1[j];
            h[j] = z[j] > 0.0 ? z[j] : 0.0;
            if (z[j] == 0.0) ++kinks;
            f += w2[j] * h[j];
        }
        double r = f - t[i];
        loss += r * r;
        double df = 2.0 * r / (double)n;
        for (int j = 0; j < 16; ++j) {
            g[32 + j] += df * h[j];
            double dz = z[j] > 0.0 ? df * w2[j] : 0.0;
            g[j] += dz * x[i];
            g[16 + j] += dz;
        }
        g[48] += df;
    }
    if (grad) std::memcpy(grad, g, sizeof g);
    if (kink) *kink = kinks;
    return n ? loss / (double)n : 0.0;
}

}  // extern "C"
