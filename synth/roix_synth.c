/*
 * roix_synth.c - seeded synthetic X-CT volumes (input generators only).
 *
 * These generators produce the test and benchmark inputs for both the CPU
 * oracle and the GPU library.  They hold none of the reduction method's
 * arithmetic: no quantisation, histogram, threshold, labelling or
 * compaction lives here.  Every value depends only on (seed, stream, voxel
 * index), so the result is bit-identical for any thread count.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written from its published
 * definition.  Normal deviates by the Box-Muller transform.
 *
 * Shapes follow the X-CT datasets of the paper's Table 1 (16-bit slice
 * stacks, cylindrical samples in air) at the sizes of the workloads:
 *   ellipsoids : background N(mu_bg, sd_bg) plus solid axis-aligned
 *                ellipsoids of intensity U(lo, hi) + N(0, sd_obj)
 *   cylinder   : z-axis cylinder (matrix) in air, with spherical pores and
 *                dense spherical inclusions; later objects overwrite
 *   rings      : uint16 z-axis cylinder, Gaussian approximation of Poisson
 *                counts, plus concentric ring artefacts constant along z
 *
 * Class maps (optional) give the analytic ground truth:
 *   ellipsoids: 0 background, e+1 for ellipsoid e (e < 254)
 *   cylinder  : 0 air, 1 matrix, 2 pore, 3 inclusion
 *   rings     : 0 outside, 1 inside the cylinder
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */

typedef struct { uint32_t v[4]; } p4x32;

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Philox4x32 with R rounds: S-box of two 32x32->64 multiplies per round,
 * Weyl-sequence key schedule. */
static p4x32 philox4x32_r(p4x32 ctr, uint32_t k0, uint32_t k1, int rounds) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int i = 0; i < rounds; ++i) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, ctr.v[0], &hi0, &lo0);
        mulhilo32(M1, ctr.v[2], &hi1, &lo1);
        p4x32 n;
        n.v[0] = hi1 ^ ctr.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ ctr.v[3] ^ k1;
        n.v[3] = lo0;
        ctr = n;
        k0 += W0;
        k1 += W1;
    }
    return ctr;
}

/* Exported for the known-answer test. */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    p4x32 c;
    memcpy(c.v, ctr, sizeof c.v);
    p4x32 r = philox4x32_r(c, key[0], key[1], 10);
    memcpy(out, r.v, sizeof r.v);
}

static inline p4x32 draw(uint64_t seed, uint32_t stream, uint64_t counter) {
    p4x32 c = {{(uint32_t)counter, (uint32_t)(counter >> 32), stream, 0u}};
    return philox4x32_r(c, (uint32_t)seed, (uint32_t)(seed >> 32), 10);
}

/* uniform double in [0,1) from 53 random bits */
static inline double u01(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return (double)m * (1.0 / 9007199254740992.0);
}

/* standard normal for voxel counter `i` of `stream` (Box-Muller, cosine branch) */
static inline double normal_at(uint64_t seed, uint32_t stream, uint64_t i) {
    p4x32 r = draw(seed, stream, i);
    double u1 = 1.0 - u01(r.v[0], r.v[1]); /* (0,1] */
    double u2 = u01(r.v[2], r.v[3]);        /* [0,1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* sequential parameter draws (object placement) */
typedef struct { uint64_t seed; uint32_t stream; uint64_t n; } pstream;
static double pnext_u01(pstream* s) {
    p4x32 r = draw(s->seed, s->stream, s->n++);
    return u01(r.v[0], r.v[1]);
}
static double pnext_uniform(pstream* s, double lo, double hi) { return lo + (hi - lo) * pnext_u01(s); }
static int64_t pnext_int(pstream* s, int64_t lo, int64_t hi_incl) {
    int64_t span = hi_incl - lo + 1;
    int64_t k = (int64_t)(pnext_u01(s) * (double)span);
    if (k >= span) k = span - 1;
    return lo + k;
}

enum { ST_NOISE = 1, ST_PARAM = 2, ST_NOISE2 = 3 };

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ------------------------------------------------------------ ellipsoids */

typedef struct {
    double cx, cy, cz, ax, ay, az, level;
} ellipsoid;

/* Fill `out` ([nz][ny][nx] float32) with the ellipsoid recipe.
 * Returns the number of ellipsoids placed (or -1 on bad arguments). */
int synth_ellipsoids_f32(float* out, uint8_t* cls, int64_t nx, int64_t ny, int64_t nz,
                         uint64_t seed, int n_ell, double mu_bg, double sd_bg,
                         double ax_lo, double ax_hi, double lev_lo, double lev_hi,
                         double sd_obj, int nthreads) {
    if (!out || nx <= 0 || ny <= 0 || nz <= 0 || n_ell < 0 || n_ell > 253) return -1;
    set_threads(nthreads);
    ellipsoid E[253];
    pstream ps = {seed, ST_PARAM, 0};
    int64_t dims[3] = {nx, ny, nz};
    for (int e = 0; e < n_ell; ++e) {
        double a[3], c[3];
        for (int k = 0; k < 3; ++k) {
            double amax = 0.5 * (double)(dims[k] - 1);
            double lo = ax_lo < amax ? ax_lo : amax, hi = ax_hi < amax ? ax_hi : amax;
            a[k] = pnext_uniform(&ps, lo, hi);
            if (a[k] < 0.5) a[k] = 0.5;
        }
        for (int k = 0; k < 3; ++k) {
            double lo = a[k], hi = (double)(dims[k] - 1) - a[k];
            c[k] = hi > lo ? pnext_uniform(&ps, lo, hi) : 0.5 * (double)(dims[k] - 1);
        }
        E[e].ax = a[0]; E[e].ay = a[1]; E[e].az = a[2];
        E[e].cx = c[0]; E[e].cy = c[1]; E[e].cz = c[2];
        E[e].level = pnext_uniform(&ps, lev_lo, lev_hi);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                int owner = -1;
                for (int e = 0; e < n_ell; ++e) {
                    double dx = ((double)x - E[e].cx) / E[e].ax;
                    double dy = ((double)y - E[e].cy) / E[e].ay;
                    double dz = ((double)z - E[e].cz) / E[e].az;
                    if (dx * dx + dy * dy + dz * dz <= 1.0) owner = e; /* later overwrite */
                }
                uint64_t v = (uint64_t)((z * ny + y) * nx + x);
                double g = normal_at(seed, ST_NOISE, v);
                double val = owner < 0 ? mu_bg + sd_bg * g : E[owner].level + sd_obj * g;
                out[v] = (float)val;
                if (cls) cls[v] = (uint8_t)(owner + 1);
            }
        }
    }
    return n_ell;
}

/* -------------------------------------------------------------- cylinder */

typedef struct { double cx, cy, cz, r; } sphere;

static sphere* place_spheres(pstream* ps, int n, double r_lo, double r_hi,
                             double ccx, double ccy, double R, int64_t nz) {
    sphere* s = (sphere*)malloc(sizeof(sphere) * (size_t)(n > 0 ? n : 1));
    if (!s) return NULL;
    for (int i = 0; i < n; ++i) {
        double r = pnext_uniform(ps, r_lo, r_hi);
        double rho_max = R - r - 1.0;
        if (rho_max < 0) rho_max = 0;
        /* uniform over the disc of radius rho_max */
        double rho = rho_max * sqrt(pnext_u01(ps));
        double th = 6.283185307179586 * pnext_u01(ps);
        s[i].cx = ccx + rho * cos(th);
        s[i].cy = ccy + rho * sin(th);
        s[i].cz = pnext_uniform(ps, 0.0, (double)(nz - 1));
        s[i].r = r;
    }
    return s;
}

static void stamp_spheres(uint8_t* c, int64_t nx, int64_t ny, int64_t z, const sphere* s, int n,
                          uint8_t label) {
    for (int i = 0; i < n; ++i) {
        double dz = (double)z - s[i].cz;
        double rr = s[i].r * s[i].r - dz * dz;
        if (rr < 0) continue;
        double h = sqrt(rr);
        int64_t y0 = (int64_t)ceil(s[i].cy - h), y1 = (int64_t)floor(s[i].cy + h);
        if (y0 < 0) y0 = 0;
        if (y1 > ny - 1) y1 = ny - 1;
        for (int64_t y = y0; y <= y1; ++y) {
            double dy = (double)y - s[i].cy;
            double r2 = rr - dy * dy;
            if (r2 < 0) continue;
            double hx = sqrt(r2);
            int64_t x0 = (int64_t)ceil(s[i].cx - hx), x1 = (int64_t)floor(s[i].cx + hx);
            if (x0 < 0) x0 = 0;
            if (x1 > nx - 1) x1 = nx - 1;
            for (int64_t x = x0; x <= x1; ++x) {
                double dx = (double)x - s[i].cx;
                if (dx * dx + dy * dy + dz * dz <= s[i].r * s[i].r) c[y * nx + x] = label;
            }
        }
    }
}

/* Cylinder sample in air.  `cls` may be NULL (then a per-thread slice buffer
 * is used).  Returns 0, or -1 on bad arguments / allocation failure. */
int synth_cylinder_f32(float* out, uint8_t* cls, int64_t nx, int64_t ny, int64_t nz, uint64_t seed,
                       double R, double mu_air, double sd_air, double mu_mat, double sd_mat,
                       int n_pores, double pr_lo, double pr_hi, double mu_pore, double sd_pore,
                       int n_incl, double ir_lo, double ir_hi, double mu_incl, double sd_incl,
                       int nthreads) {
    if (!out || nx <= 0 || ny <= 0 || nz <= 0 || n_pores < 0 || n_incl < 0) return -1;
    set_threads(nthreads);
    double ccx = 0.5 * (double)nx, ccy = 0.5 * (double)ny;
    pstream ps = {seed, ST_PARAM, 0};
    sphere* P = place_spheres(&ps, n_pores, pr_lo, pr_hi, ccx, ccy, R, nz);
    sphere* I = place_spheres(&ps, n_incl, ir_lo, ir_hi, ccx, ccy, R, nz);
    if (!P || !I) { free(P); free(I); return -1; }
    int fail = 0;
#pragma omp parallel
    {
        uint8_t* slice = (uint8_t*)malloc((size_t)(nx * ny));
        if (!slice) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t z = 0; z < nz; ++z) {
            if (!slice) continue;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    double dx = (double)x - ccx, dy = (double)y - ccy;
                    slice[y * nx + x] = (dx * dx + dy * dy <= R * R) ? 1 : 0;
                }
            stamp_spheres(slice, nx, ny, z, P, n_pores, 2);
            stamp_spheres(slice, nx, ny, z, I, n_incl, 3);
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    uint64_t v = (uint64_t)((z * ny + y) * nx + x);
                    uint8_t k = slice[y * nx + x];
                    double g = normal_at(seed, ST_NOISE, v), val;
                    switch (k) {
                        case 0: val = mu_air + sd_air * g; break;
                        case 1: val = mu_mat + sd_mat * g; break;
                        case 2: val = mu_pore + sd_pore * g; break;
                        default: val = mu_incl + sd_incl * g; break;
                    }
                    out[v] = (float)val;
                    if (cls) cls[v] = k;
                }
        }
        free(slice);
    }
    free(P);
    free(I);
    return fail ? -1 : 0;
}

/* ----------------------------------------------------------------- rings */

/* uint16 cylinder with ring artefacts.  lambda(x,y) = lam_in inside radius R,
 * lam_out outside, plus `offset` for every ring whose [radius, radius+width)
 * contains the voxel's radial distance.  Value = clamp(rint(lambda +
 * sqrt(lambda) * N(0,1)), 0, 65535). */
/* Planes [z0, z0 + nz) of that volume (the noise counter is the voxel's
 * linear index in the whole volume, so slabs cut this way assemble into
 * exactly the volume synth_rings_u16 writes). */
int synth_rings_u16_planes(uint16_t* out, uint8_t* cls, int64_t nx, int64_t ny, int64_t z0, int64_t nz,
                           uint64_t seed, double R, double lam_in, double lam_out, int n_rings, double ring_rmax,
                           double ring_amp, int nthreads) {
    if (!out || nx <= 0 || ny <= 0 || nz <= 0 || z0 < 0 || n_rings < 0) return -1;
    set_threads(nthreads);
    double ccx = 0.5 * (double)nx, ccy = 0.5 * (double)ny;
    double* rr = (double*)malloc(sizeof(double) * (size_t)(n_rings > 0 ? n_rings : 1));
    double* rw = (double*)malloc(sizeof(double) * (size_t)(n_rings > 0 ? n_rings : 1));
    double* ra = (double*)malloc(sizeof(double) * (size_t)(n_rings > 0 ? n_rings : 1));
    float* lam = (float*)malloc(sizeof(float) * (size_t)(nx * ny));
    uint8_t* inside = (uint8_t*)malloc((size_t)(nx * ny));
    if (!rr || !rw || !ra || !lam || !inside) {
        free(rr); free(rw); free(ra); free(lam); free(inside);
        return -1;
    }
    pstream ps = {seed, ST_PARAM, 0};
    for (int i = 0; i < n_rings; ++i) {
        rr[i] = pnext_uniform(&ps, 0.0, ring_rmax);
        rw[i] = (double)pnext_int(&ps, 1, 3);
        ra[i] = pnext_u01(&ps) < 0.5 ? -ring_amp : ring_amp;
    }
    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            double dx = (double)x - ccx, dy = (double)y - ccy;
            double rho = sqrt(dx * dx + dy * dy);
            int in = dx * dx + dy * dy <= R * R;
            double l = in ? lam_in : lam_out;
            for (int i = 0; i < n_rings; ++i)
                if (rho >= rr[i] && rho < rr[i] + rw[i]) l += ra[i];
            lam[y * nx + x] = (float)l;
            inside[y * nx + x] = (uint8_t)in;
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t p = 0; p < nx * ny; ++p) {
            uint64_t v = (uint64_t)(z * nx * ny + p);
            double l = (double)lam[p];
            double val = rint(l + sqrt(l) * normal_at(seed, ST_NOISE, v + (uint64_t)(z0 * nx * ny)));
            if (val < 0) val = 0;
            if (val > 65535) val = 65535;
            out[v] = (uint16_t)val;
            if (cls) cls[v] = inside[p];
        }
    }
    free(rr); free(rw); free(ra); free(lam); free(inside);
    return 0;
}

int synth_rings_u16(uint16_t* out, uint8_t* cls, int64_t nx, int64_t ny, int64_t nz, uint64_t seed,
                    double R, double lam_in, double lam_out, int n_rings, double ring_rmax,
                    double ring_amp, int nthreads) {
    return synth_rings_u16_planes(out, cls, nx, ny, 0, nz, seed, R, lam_in, lam_out, n_rings, ring_rmax,
                                  ring_amp, nthreads);
}

/* Uniform random bytes (for tiny adversarial test masks); byte v is 1 with
 * probability p, else 0. */
void synth_bernoulli_u8(uint8_t* out, int64_t n, uint64_t seed, double p) {
    for (int64_t v = 0; v < n; ++v) {
        p4x32 r = draw(seed, ST_NOISE2, (uint64_t)v);
        out[v] = u01(r.v[0], r.v[1]) < p ? 1 : 0;
    }
}

/* Normal deviates (used by tests that need plain noise volumes). */
void synth_normal_f32(float* out, int64_t n, uint64_t seed, double mu, double sd, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) out[v] = (float)(mu + sd * normal_at(seed, ST_NOISE, (uint64_t)v));
}
