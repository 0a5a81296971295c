/*
 * Seeded synthetic point-cloud generators.
 *
 * These stand in for the datasets the paper evaluates on (8i voxelized
 * surface light fields and Paris-Lille-3 LiDAR, Section VI-B), which are not
 * available.  They produce float32 xyz clouds, query points and random index
 * sets only; they contain none of the CGA arithmetic (no quantization, key
 * encoding, sorting, set operations or searches), so both the GPU path and the
 * CPU oracle can consume them without sharing any of the method.
 *
 * Every quantity is computed in double and rounded to float32 once.
 * Randomness: splitmix64 seeding of xoshiro256** (Blackman & Vigna), normals
 * by Box-Muller.  Each point draws from its own stream keyed by
 * (seed, stream, index), so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void rng_init(rng_t *r, uint64_t seed, uint64_t stream, uint64_t index) {
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ull) ^ (index * 0x8CB92BA72F3D8DD7ull);
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
static double rng_uniform(rng_t *r, double lo, double hi) { return lo + (hi - lo) * rng_u01(r); }

static double rng_normal(rng_t *r) {
    double u1 = rng_u01(r), u2 = rng_u01(r);
    if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

static void rng_unit_vector(rng_t *r, double v[3]) {
    double n;
    do {
        v[0] = rng_normal(r); v[1] = rng_normal(r); v[2] = rng_normal(r);
        n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    } while (n < 1e-12);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/* ------------------------------------------------------------------ */
/* Spheres: points on the surfaces of random spheres in the unit cube. */
/* ------------------------------------------------------------------ */

/* Writes n points to a (float32 AoS).  If b is non-NULL it also writes a copy
 * of the same (double) points rotated by rot_deg about the z axis through
 * (pivot_x, pivot_y) and shifted by (shift_x, 0, 0).  */
void gen_spheres(uint64_t seed, int64_t n, int nsph, double jitter,
                 double rot_deg, double pivot_x, double pivot_y, double shift_x,
                 float *a, float *b) {
    double c[64][3], rad[64], cum[65];
    rng_t r;
    rng_init(&r, seed, 0, 0);
    if (nsph > 64) nsph = 64;
    cum[0] = 0.0;
    for (int s = 0; s < nsph; ++s) {
        for (int k = 0; k < 3; ++k) c[s][k] = rng_uniform(&r, 0.2, 0.8);
        rad[s] = rng_uniform(&r, 0.05, 0.2);
        cum[s + 1] = cum[s] + rad[s] * rad[s];
    }
    const double th = rot_deg * M_PI / 180.0, ct = cos(th), st = sin(th);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, 1, (uint64_t)i);
        double pick = rng_u01(&q) * cum[nsph];
        int s = 0;
        while (s < nsph - 1 && pick >= cum[s + 1]) ++s;
        double d[3];
        rng_unit_vector(&q, d);
        double p[3];
        for (int k = 0; k < 3; ++k) p[k] = c[s][k] + rad[s] * d[k] + jitter * rng_normal(&q);
        a[3 * i + 0] = (float)p[0];
        a[3 * i + 1] = (float)p[1];
        a[3 * i + 2] = (float)p[2];
        if (b) {
            double x = p[0] - pivot_x, y = p[1] - pivot_y;
            b[3 * i + 0] = (float)(pivot_x + ct * x - st * y + shift_x);
            b[3 * i + 1] = (float)(pivot_y + st * x + ct * y);
            b[3 * i + 2] = (float)p[2];
        }
    }
}

/* Uniform points in the axis-aligned box [lo, hi). */
void gen_uniform_box(uint64_t seed, uint64_t stream, int64_t n, const double lo[3],
                     const double hi[3], float *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, stream, (uint64_t)i);
        for (int k = 0; k < 3; ++k) out[3 * i + k] = (float)rng_uniform(&q, lo[k], hi[k]);
    }
}

/* ------------------------------------------------------------------ */
/* Gaussian-bump-perturbed unit sphere ("graphics model").             */
/* ------------------------------------------------------------------ */
void gen_bumpy_sphere(uint64_t seed, int64_t n, int nbumps, double rot_deg,
                      float *a, float *b) {
    double c[256][3], amp[256], w[256];
    rng_t r;
    rng_init(&r, seed, 0, 0);
    if (nbumps > 256) nbumps = 256;
    for (int j = 0; j < nbumps; ++j) {
        rng_unit_vector(&r, c[j]);
        amp[j] = rng_uniform(&r, 0.0, 0.1);
        w[j] = rng_uniform(&r, 0.05, 0.3);
    }
    const double th = rot_deg * M_PI / 180.0, ct = cos(th), st = sin(th);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, 1, (uint64_t)i);
        double u[3];
        rng_unit_vector(&q, u);
        double rr = 1.0;
        for (int j = 0; j < nbumps; ++j) {
            double dx = u[0] - c[j][0], dy = u[1] - c[j][1], dz = u[2] - c[j][2];
            double d2 = dx * dx + dy * dy + dz * dz;
            rr += amp[j] * exp(-d2 / (2.0 * w[j] * w[j]));
        }
        double p[3] = {rr * u[0], rr * u[1], rr * u[2]};
        a[3 * i + 0] = (float)p[0];
        a[3 * i + 1] = (float)p[1];
        a[3 * i + 2] = (float)p[2];
        if (b) {
            b[3 * i + 0] = (float)(ct * p[0] - st * p[1]);
            b[3 * i + 1] = (float)(st * p[0] + ct * p[1]);
            b[3 * i + 2] = (float)p[2];
        }
    }
}

/* ------------------------------------------------------------------ */
/* LiDAR-like scene: ground plane z = 0 plus axis-aligned boxes.       */
/* A box is 6 doubles: xmin, ymin, zmin(=0), xmax, ymax, zmax.         */
/* ------------------------------------------------------------------ */
void gen_lidar_scene(uint64_t seed, int nboxes, double half_extent, double clear_x0,
                     double clear_x1, double *boxes) {
    rng_t r;
    rng_init(&r, seed, 0, 0);
    for (int i = 0; i < nboxes; ++i) {
        for (;;) {
            double cx = rng_uniform(&r, -half_extent, half_extent);
            double cy = rng_uniform(&r, -half_extent, half_extent);
            double sx = rng_uniform(&r, 1.0, 8.0), sy = rng_uniform(&r, 1.0, 8.0);
            double h = rng_uniform(&r, 0.5, 4.0);
            /* keep a 4 m clearance between every box footprint and the sensor
             * positions on the segment (clear_x0..clear_x1, 0) */
            double nx = cx < clear_x0 ? clear_x0 : (cx > clear_x1 ? clear_x1 : cx);
            double dx = fabs(cx - nx) - sx / 2, dy = fabs(cy) - sy / 2;
            if (dx < 0) dx = 0;
            if (dy < 0) dy = 0;
            if (dx * dx + dy * dy < 16.0) continue;
            boxes[6 * i + 0] = cx - sx / 2; boxes[6 * i + 1] = cy - sy / 2; boxes[6 * i + 2] = 0.0;
            boxes[6 * i + 3] = cx + sx / 2; boxes[6 * i + 4] = cy + sy / 2; boxes[6 * i + 5] = h;
            break;
        }
    }
}

/* One sweep: `rings` elevations evenly spaced in [el_lo, el_hi] degrees,
 * `naz` azimuth steps starting at `yaw` (degrees), sensor at `pose` (x, y, z).
 * Each ray's range is its first hit (ground or box, slab test) plus
 * N(0, sigma^2) noise from stream `stream`.  Writes rings*naz points. */
void gen_lidar_sweep(uint64_t seed, uint64_t stream, const double *boxes, int nboxes,
                     const double pose[3], double yaw_deg, int rings, int64_t naz,
                     double el_lo, double el_hi, double sigma, float *out) {
    const int64_t total = (int64_t)rings * naz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < total; ++i) {
        int ring = (int)(i / naz);
        int64_t az = i % naz;
        double el = (rings > 1 ? el_lo + (el_hi - el_lo) * ring / (rings - 1) : el_lo) * M_PI / 180.0;
        double a = yaw_deg * M_PI / 180.0 + 2.0 * M_PI * (double)az / (double)naz;
        double d[3] = {cos(el) * cos(a), cos(el) * sin(a), sin(el)};
        double t = d[2] < 0 ? -pose[2] / d[2] : 1e9;
        for (int bx = 0; bx < nboxes; ++bx) {
            const double *B = boxes + 6 * bx;
            double t0 = -1e300, t1 = 1e300;
            int miss = 0;
            for (int k = 0; k < 3 && !miss; ++k) {
                if (fabs(d[k]) < 1e-15) {
                    if (pose[k] < B[k] || pose[k] > B[k + 3]) miss = 1;
                } else {
                    double ta = (B[k] - pose[k]) / d[k], tb = (B[k + 3] - pose[k]) / d[k];
                    if (ta > tb) { double s = ta; ta = tb; tb = s; }
                    if (ta > t0) t0 = ta;
                    if (tb < t1) t1 = tb;
                }
            }
            if (miss || t0 > t1 || t0 <= 0.0) continue; /* no hit, or sensor inside */
            if (t0 < t) t = t0;
        }
        rng_t q;
        rng_init(&q, seed, stream, (uint64_t)i);
        double range = t + sigma * rng_normal(&q);
        out[3 * i + 0] = (float)(pose[0] + range * d[0]);
        out[3 * i + 1] = (float)(pose[1] + range * d[1]);
        out[3 * i + 2] = (float)(pose[2] + range * d[2]);
    }
}

/* Random-walk poses: frame f+1 = frame f moved `step` in a uniform random
 * heading, yaw changed by U[-yaw_step, yaw_step] degrees.  Writes x, y, z, yaw
 * per frame.  Also draws per-frame sizes n_f = floor(exp(U[ln lo, ln hi]))
 * when sizes is non-NULL. */
void gen_random_walk(uint64_t seed, int nframes, const double start[3], double step,
                     double yaw_step, double size_lo, double size_hi, double *poses,
                     int64_t *sizes) {
    rng_t r;
    rng_init(&r, seed, 7, 0);
    double x = start[0], y = start[1], yaw = 0.0;
    for (int f = 0; f < nframes; ++f) {
        poses[4 * f + 0] = x; poses[4 * f + 1] = y; poses[4 * f + 2] = start[2]; poses[4 * f + 3] = yaw;
        if (sizes) sizes[f] = (int64_t)floor(exp(rng_uniform(&r, log(size_lo), log(size_hi))));
        double h = rng_uniform(&r, 0.0, 2.0 * M_PI);
        x += step * cos(h);
        y += step * sin(h);
        yaw += rng_uniform(&r, -yaw_step, yaw_step);
    }
}

/* Points near a cloud: out[i] = src[idx] + N(0, sigma^2 I), idx uniform. */
void gen_jittered_picks(uint64_t seed, uint64_t stream, const float *src, int64_t nsrc,
                        int64_t n, double sigma, float *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, stream, (uint64_t)i);
        int64_t j = (int64_t)(rng_next(&q) % (uint64_t)nsrc);
        for (int k = 0; k < 3; ++k) out[3 * i + k] = (float)((double)src[3 * j + k] + sigma * rng_normal(&q));
    }
}

/* Uniform random integers in [0, m): out[i] for i < n. */
void gen_uniform_index(uint64_t seed, uint64_t stream, int64_t n, uint64_t m, int64_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, stream, (uint64_t)i);
        out[i] = (int64_t)(rng_next(&q) % m);
    }
}

/* Uniform random u64 in [lo, hi]. */
void gen_uniform_u64(uint64_t seed, uint64_t stream, int64_t n, uint64_t lo, uint64_t hi,
                     uint64_t *out) {
    uint64_t span = hi - lo + 1; /* span == 0 means the full 2^64 range */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t q;
        rng_init(&q, seed, stream, (uint64_t)i);
        uint64_t v = rng_next(&q);
        out[i] = span ? lo + v % span : v;
    }
}

/* Sorted uniform random subset of size m from {0..u-1} (selection sampling,
 * Knuth TAOCP vol. 2, Algorithm 3.4.2 S).  Returns the number written. */
int64_t gen_subset(uint64_t seed, int64_t u, int64_t m, int64_t *out) {
    rng_t r;
    rng_init(&r, seed, 9, 0);
    int64_t chosen = 0;
    for (int64_t t = 0; t < u && chosen < m; ++t) {
        double v = rng_u01(&r);
        if ((double)(u - t) * v < (double)(m - chosen)) out[chosen++] = t;
    }
    return chosen;
}

/* Fisher-Yates permutation of out[0..n) in place. */
void gen_shuffle_i64(uint64_t seed, int64_t n, int64_t *out) {
    rng_t r;
    rng_init(&r, seed, 11, 0);
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)(rng_next(&r) % (uint64_t)(i + 1));
        int64_t t = out[i]; out[i] = out[j]; out[j] = t;
    }
}

/* Raw xoshiro256** outputs of stream (seed, stream, index), for tests. */
void gen_raw(uint64_t seed, uint64_t stream, uint64_t index, int n, uint64_t *out) {
    rng_t r;
    rng_init(&r, seed, stream, index);
    for (int i = 0; i < n; ++i) out[i] = rng_next(&r);
}

/* Seeded per-point attributes: four 8-bit channels packed in a uint32
 * (channel c in bits 8c .. 8c + 7), uniform, one draw per point from stream
 * (seed, stream, point index). */
void gen_attributes(uint64_t seed, uint64_t stream, int64_t n, uint32_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rng_t r;
        rng_init(&r, seed, stream, (uint64_t)i);
        out[i] = (uint32_t)(rng_next(&r) >> 32);
    }
}
