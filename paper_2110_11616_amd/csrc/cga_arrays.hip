// The paper's own operations on the five coordinate arrays of a LINEAR CGA
// (X_index, X_pointer, Y_index, Y_pointer, Z_index; Section V), one thread
// per lookup and a team of lanes per nearest-neighbour query:
//
// * point lookup, Section V-A: the query's x is searched in X_index, its
//   X_pointer entries bound the run of Y_index holding that x's y values,
//   the query's y is searched there, its Y_pointer entries bound the run of
//   Z_index holding that (x, y)'s z values, and the query's z is searched
//   there.  X_pointer is indexed by the position of the x in X_index.
//
// * nearest neighbour, Section V-C: the nearest x in X_index, then the
//   nearest y in its run, then the nearest z in that run give a first point
//   at distance epsilon (0 for an exact match); the answer is the closest
//   point whose coordinates all lie within epsilon of the query's.  The box
//   is walked x by x and y by y in ascending order, each range found by a
//   search and narrowed as closer points turn up, and only the nearest z
//   below and at-or-above the query's is tried in each (x, y) run (every other
//   z of the run is farther); ties go to the smaller position, i.e. the
//   smaller LINEAR key, as in every other k-NN of this library.
//
// Pointers are checked against the array lengths as they are read, so that
// arrays that are not a CGA keep every access in bounds (ERR_MISMATCH).
#include "cga_common.h"

namespace cga {

// First index in [lo, hi) of an ascending run whose value is >= v.
__device__ __forceinline__ int64_t run_lower(const uint32_t *__restrict__ a, int64_t lo, int64_t hi,
                                             uint32_t v) {
    int64_t len = hi - lo;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (a[lo + half] < v) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// Index in the non-empty run [lo, hi) of the value closest to v (the smaller
// value on a tie).
__device__ __forceinline__ int64_t run_nearest(const uint32_t *__restrict__ a, int64_t lo, int64_t hi,
                                               uint32_t v) {
    const int64_t p = run_lower(a, lo, hi, v);
    if (p == hi) return hi - 1;
    if (p == lo) return lo;
    return v - a[p - 1] <= a[p] - v ? p - 1 : p;
}

__device__ __forceinline__ uint64_t sq_gap(uint32_t a, uint32_t b) {
    const uint64_t d = a > b ? a - b : b - a;
    return d * d;
}

__device__ __forceinline__ uint32_t isqrt_u64(uint64_t v) {
    uint64_t r = (uint64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (uint32_t)r;
}

// The five arrays with their lengths: host bounds, lowered to the device
// counts (when given) by resolve() inside the kernel.
struct Arrays {
    const uint32_t *xi;
    const int64_t *xp;
    const uint32_t *yi;
    const int64_t *yp;
    const uint32_t *zi;
    int64_t nx, nxy, n;
    const int64_t *d_nx, *d_nxy;
    uint32_t *err;

    __device__ __forceinline__ void resolve() {
        const int64_t cx = dev_count(nx, d_nx), cxy = dev_count(nxy, d_nxy);
        nx = cx < nx ? cx : nx;
        nxy = cxy < nxy ? cxy : nxy;
    }

    // Run [lo, hi) of Y_index for X_index entry a, clamped to the array.
    __device__ __forceinline__ void y_run(int64_t a, int64_t &lo, int64_t &hi) const {
        lo = xp[a];
        hi = xp[a + 1];
        fix(lo, hi, nxy);
    }
    __device__ __forceinline__ void z_run(int64_t b, int64_t &lo, int64_t &hi) const {
        lo = yp[b];
        hi = yp[b + 1];
        fix(lo, hi, n);
    }
    __device__ __forceinline__ void fix(int64_t &lo, int64_t &hi, int64_t len) const {
        if (lo < 0 || hi < lo || hi > len) {
            set_err(err, ERR_MISMATCH);
            lo = lo < 0 ? 0 : (lo > len ? len : lo);
            hi = hi < lo ? lo : (hi > len ? len : hi);
        }
    }
};

__global__ __launch_bounds__(256) void k_arrays_lookup(Arrays A, const uint32_t *__restrict__ qvox,
                                                       int64_t nq, int64_t *__restrict__ pos) {
    A.resolve();
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nq;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t qx = qvox[3 * j], qy = qvox[3 * j + 1], qz = qvox[3 * j + 2];
        int64_t p = -1;
        const int64_t a = run_lower(A.xi, 0, A.nx, qx);
        if (a < A.nx && A.xi[a] == qx) {
            int64_t b0, b1;
            A.y_run(a, b0, b1);
            const int64_t b = run_lower(A.yi, b0, b1, qy);
            if (b < b1 && A.yi[b] == qy) {
                int64_t c0, c1;
                A.z_run(b, c0, c1);
                const int64_t c = run_lower(A.zi, c0, c1, qz);
                if (c < c1 && A.zi[c] == qz) p = c;
            }
        }
        pos[j] = p;
    }
}

// Nearest neighbour, a team of kNnTeam lanes per query.  Every lane finds
// the same first point; then lane t walks the x entries a0 + t, a0 + t +
// kNnTeam, ... of the box, keeping its own best and pruning against the
// smallest distance found so far by any lane of the team (an LDS word).  A
// pruned point is strictly farther than a point already found, so every
// point at the final distance is still examined, and the lexicographic
// minimum of (squared distance, position) over the lanes is the answer of
// the one-lane walk.
constexpr int kNnTeam = 8;
constexpr int kNnBlock = 256;

__global__ __launch_bounds__(kNnBlock) void k_arrays_nn(Arrays A, const float *__restrict__ q,
                                                        int64_t nq, float o0, float o1, float o2,
                                                        float scale, uint32_t depth,
                                                        int64_t *__restrict__ idx,
                                                        uint64_t *__restrict__ d2) {
    __shared__ unsigned long long s_bd[kNnBlock / kNnTeam];
    A.resolve();
    const float o[3] = {o0, o1, o2};
    const int team = threadIdx.x / kNnTeam, tl = threadIdx.x % kNnTeam;
    const int64_t teams = (int64_t)gridDim.x * (kNnBlock / kNnTeam);
    // j is the same for the kNnTeam lanes of a team, so the team stays together
    for (int64_t j = (int64_t)blockIdx.x * (kNnBlock / kNnTeam) + team; j < nq; j += teams) {
        Vox v;
        if (!quantize3(q[3 * j], q[3 * j + 1], q[3 * j + 2], o, scale, depth, v)) {
            if (tl == 0) {
                set_err(A.err, ERR_NONFINITE);
                idx[j] = -1;
                d2[j] = ~0ull;
            }
            continue;
        }
        int64_t best = -1;
        uint64_t bd = ~0ull;
        // first point: nearest x, then nearest y in its run, nearest z in that run
        if (A.nx > 0) {
            const int64_t a = run_nearest(A.xi, 0, A.nx, v.x);
            int64_t b0, b1, c0, c1;
            A.y_run(a, b0, b1);
            if (b0 < b1) {
                const int64_t b = run_nearest(A.yi, b0, b1, v.y);
                A.z_run(b, c0, c1);
                if (c0 < c1) {
                    const int64_t c = run_nearest(A.zi, c0, c1, v.z);
                    best = c;
                    bd = sq_gap(A.xi[a], v.x) + sq_gap(A.yi[b], v.y) + sq_gap(A.zi[c], v.z);
                }
            }
        }
        if (best >= 0 && bd > 0) {
            s_bd[team] = bd;  // every lane stores the same value
            // the box |coordinate - query| <= epsilon, narrowed as the team's bound falls
            const uint32_t e = isqrt_u64(bd);
            const int64_t a0 = run_lower(A.xi, 0, A.nx, v.x > e ? v.x - e : 0);
            for (int64_t a = a0 + tl; a < A.nx; a += kNnTeam) {
                uint64_t B = __hip_atomic_load(&s_bd[team], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                B = bd < B ? bd : B;
                const uint32_t x = A.xi[a];
                const uint64_t dx2 = sq_gap(x, v.x);
                if (dx2 > B) {
                    if (x > v.x) break;
                    continue;
                }
                int64_t b0, b1;
                A.y_run(a, b0, b1);
                const uint32_t ey = isqrt_u64(B - dx2);
                for (int64_t b = run_lower(A.yi, b0, b1, v.y > ey ? v.y - ey : 0); b < b1; ++b) {
                    const uint32_t y = A.yi[b];
                    const uint64_t dxy = dx2 + sq_gap(y, v.y);
                    if (dxy > B) {
                        if (y > v.y) break;
                        continue;
                    }
                    int64_t c0, c1;
                    A.z_run(b, c0, c1);
                    const int64_t p = run_lower(A.zi, c0, c1, v.z);
                    if (p > c0) {  // nearest z below the query's
                        const uint64_t d = dxy + sq_gap(A.zi[p - 1], v.z);
                        if (d < bd || (d == bd && p - 1 < best)) {
                            bd = d;
                            best = p - 1;
                        }
                    }
                    if (p < c1) {  // nearest z at or above it
                        const uint64_t d = dxy + sq_gap(A.zi[p], v.z);
                        if (d < bd || (d == bd && p < best)) {
                            bd = d;
                            best = p;
                        }
                    }
                    if (bd < B) {
                        B = bd;
                        atomicMin(&s_bd[team], (unsigned long long)bd);
                    }
                }
            }
        }
        // lexicographic minimum of (bd, best) over the team
#pragma unroll
        for (int m = 1; m < kNnTeam; m <<= 1) {
            const uint64_t ob = __shfl_xor(bd, m, kNnTeam);
            const int64_t op = __shfl_xor(best, m, kNnTeam);
            if (ob < bd || (ob == bd && op < best)) {
                bd = ob;
                best = op;
            }
        }
        if (tl == 0) {
            idx[j] = best;
            d2[j] = bd;
        }
    }
}

static unsigned arrays_grid(int64_t nq) {
    int64_t b = (nq + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

static bool arrays_args_ok(const cga_grid *g, const uint32_t *xi, int64_t nx, const int64_t *xp,
                           const uint32_t *yi, int64_t nxy, const int64_t *yp, const uint32_t *zi,
                           int64_t n) {
    if (!grid_valid(g) || nx < 0 || nxy < 0 || n < 0 || !xp || !yp) return false;
    return !((nx > 0 && !xi) || (nxy > 0 && !yi) || (n > 0 && !zi));
}

}  // namespace cga

using namespace cga;

extern "C" {

size_t cga_arrays_ops_workspace_bytes(void) { return kControlBytes; }

int cga_arrays_lookup(const cga_grid *g, const uint32_t *d_x_index, int64_t n_x,
                      const int64_t *d_n_x, const int64_t *d_x_ptr, const uint32_t *d_y_index,
                      int64_t n_xy, const int64_t *d_n_xy, const int64_t *d_y_ptr,
                      const uint32_t *d_z_index, int64_t n, const uint32_t *d_qvox, int64_t nq,
                      int64_t *d_pos, void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!arrays_args_ok(g, d_x_index, n_x, d_x_ptr, d_y_index, n_xy, d_y_ptr, d_z_index, n) ||
        nq < 0 || !d_ws)
        return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_LINEAR) return CGA_EMISMATCH;
    if (nq > 0 && (!d_qvox || !d_pos)) return CGA_EINVAL;
    if (ws_bytes < cga_arrays_ops_workspace_bytes()) return CGA_EWORKSPACE;
    Control *ctl = (Control *)d_ws;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (nq > 0) {
        CGA_PROF("arrays_lookup", s);
        const Arrays A{d_x_index, d_x_ptr, d_y_index, d_y_ptr, d_z_index, n_x, n_xy, n,
                       d_n_x, d_n_xy, &ctl->err};
        k_arrays_lookup<<<arrays_grid(nq), 256, 0, s>>>(A, d_qvox, nq, d_pos);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

int cga_arrays_nn(const cga_grid *g, const uint32_t *d_x_index, int64_t n_x, const int64_t *d_n_x,
                  const int64_t *d_x_ptr, const uint32_t *d_y_index, int64_t n_xy,
                  const int64_t *d_n_xy, const int64_t *d_y_ptr, const uint32_t *d_z_index,
                  int64_t n, const float *d_q, int64_t nq, int64_t *d_idx, uint64_t *d_d2,
                  void *d_ws, size_t ws_bytes, cga_stream stream) {
    if (!arrays_args_ok(g, d_x_index, n_x, d_x_ptr, d_y_index, n_xy, d_y_ptr, d_z_index, n) ||
        nq < 0 || !d_ws)
        return CGA_EINVAL;
    if (g->key_mode != CGA_KEY_LINEAR) return CGA_EMISMATCH;
    if (nq > 0 && (!d_q || !d_idx || !d_d2)) return CGA_EINVAL;
    if (ws_bytes < cga_arrays_ops_workspace_bytes()) return CGA_EWORKSPACE;
    Control *ctl = (Control *)d_ws;
    hipStream_t s = (hipStream_t)stream;
    CGA_TRY(launch_begin(ctl, nullptr, 0, nullptr, 0, nullptr, s));
    if (nq > 0) {
        CGA_PROF("arrays_nn", s);
        const Arrays A{d_x_index, d_x_ptr, d_y_index, d_y_ptr, d_z_index, n_x, n_xy, n,
                       d_n_x, d_n_xy, &ctl->err};
        k_arrays_nn<<<arrays_grid(nq * kNnTeam), kNnBlock, 0, s>>>(
            A, d_q, nq, g->origin[0], g->origin[1], g->origin[2], g->scale, g->depth, d_idx, d_d2);
    }
    CGA_HIP(hipGetLastError());
    return CGA_OK;
}

}  // extern "C"
