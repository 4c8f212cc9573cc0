/*
 * scenegen.c -- seeded synthetic participating media and an instrumented
 * delta-tracking volume path tracer.
 *
 * This is the INPUT side of the project. It produces, in path order, the
 * per-scattering-vertex records that the path-graph method consumes: the
 * collision position, the arriving and the phase-sampled continuation
 * directions, the next-event (emitter-sampling) records and the radiance that
 * reached the vertex along its own continuation when that ray escaped (paper,
 * Sec. "Volume Path Tracing" and the "Instrumented path tracer" paragraph of
 * Sec. "Rendering System").  It holds none of the path-graph arithmetic: no
 * neighbour search, no MIS weights, no aggregation and no propagation.  Both
 * the FP64 oracle and the GPU library read what it writes.
 *
 * Medium: unit cube [0,1]^3, density grid R^3 (nearest voxel), vacuum outside.
 *   sigma_t = sigma_max * clamp(0.5 + c (fbm(x) - 0.5) + b, 0, 1) [* soft sphere
 *   mask]; fbm = 4 octaves of value noise, base lattice frequency 4,
 *   lacunarity 2, gain 0.5, smoothstep interpolation, normalised by the
 *   amplitude sum (so fbm lies in [0,1]); contrast c and bias b shape it.
 * Albedo: constant, or per voxel uniform in [lo, hi] (hashed per voxel).  The
 *   albedo is a throughput weight only; path geometry never depends on it, so
 *   "paths held fixed" is exact when albedo changes.
 * Lights: one directional (delta) sun and a constant environment.
 * Tracer: analog delta tracking against the grid-maximum majorant; at every
 *   collision vertex a sun shadow ray and one uniform-sphere environment shadow
 *   ray, both with ratio-tracking transmittance; the continuation direction is
 *   sampled from Henyey-Greenstein with parameter g about the arriving
 *   direction.  At most max_depth vertices per path; the last one gets no
 *   continuation (its escaped-radiance record is 0).  No Russian roulette.
 * Random numbers: PCG32 (O'Neill 2014, pcg32_random_r), one stream per pixel
 *   of the full image, seeded by (scene seed, sample index).  A crop of the
 *   image therefore traces exactly the same paths as the full image does at
 *   those pixels and samples.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -ffp-contract=off scenegen.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct sg_config {
    int32_t R;              /* density grid resolution per axis */
    int32_t mask;           /* 0: none, 1: soft sphere 1 - smoothstep(r0, r1, |x - c|) */
    int32_t albedo_mode;    /* 0: constant albedo_lo, 1: per-voxel U[albedo_lo, albedo_hi] */
    int32_t width, height;  /* full image size */
    int32_t spp;
    int32_t max_depth;      /* maximum number of scattering vertices per path */
    int32_t crop_x0, crop_y0, crop_w, crop_h; /* traced window; crop_w == 0: full image */
    int32_t pad_;
    double sigma_max;
    double density_contrast, density_bias; /* n' = clamp(0.5 + c (n - 0.5) + b, 0, 1) */
    double mask_r0, mask_r1;
    double albedo_lo, albedo_hi;
    double g;               /* HG parameter used to sample continuation directions */
    double cam_pos[3], look_at[3], vfov_deg;
    double sun_dir[3];      /* unit vector pointing toward the sun */
    double sun_E[3];        /* sun irradiance (RGB) */
    double env_L[3];        /* constant environment radiance (RGB) */
    uint64_t seed;
    int32_t extra_samples;  /* extra emitter samples at each path's first vertex */
    int32_t point_light;    /* 1: a point light at pl_pos with intensity pl_I */
    double pl_pos[3];
    double pl_I[3];
} sg_config;

/* ------------------------------------------------------------------ RNG --- */
typedef struct { uint64_t state, inc; } pcg32;

static uint32_t pcg32_next(pcg32* r) {
    uint64_t old = r->state;
    r->state = old * 6364136223846793005ULL + r->inc;
    uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
    uint32_t rot = (uint32_t)(old >> 59u);
    return (xs >> rot) | (xs << ((-rot) & 31u));
}
static void pcg32_seed(pcg32* r, uint64_t initstate, uint64_t initseq) {
    r->state = 0u;
    r->inc = (initseq << 1u) | 1u;
    pcg32_next(r);
    r->state += initstate;
    pcg32_next(r);
}
/* uniform double in [0,1) with 32 random bits */
static double rnd(pcg32* r) { return (double)pcg32_next(r) * (1.0 / 4294967296.0); }

static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}
/* 32-bit integer finaliser ("lowbias32", C. Wellons) */
static uint32_t hash32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}
static double hash_unit(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
    uint32_t h = hash32(a ^ 0x68e31da4U);
    h = hash32(h ^ b); h = hash32(h ^ c); h = hash32(h ^ d); h = hash32(h ^ e);
    return (double)(h >> 8) * (1.0 / 16777216.0);
}

/* --------------------------------------------------------------- medium --- */
static double smooth01(double t) { return t * t * (3.0 - 2.0 * t); }
static double smoothstep(double e0, double e1, double x) {
    double t = (x - e0) / (e1 - e0);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    return smooth01(t);
}

static double value_noise(uint32_t seed, int oct, double px, double py, double pz) {
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    double tx = smooth01(px - fx), ty = smooth01(py - fy), tz = smooth01(pz - fz);
    double v[2][2][2];
    for (int c = 0; c < 8; ++c) {
        int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        v[dz][dy][dx] = hash_unit(seed, (uint32_t)oct, (uint32_t)(ix + dx), (uint32_t)(iy + dy), (uint32_t)(iz + dz));
    }
    double x00 = v[0][0][0] + (v[0][0][1] - v[0][0][0]) * tx;
    double x10 = v[0][1][0] + (v[0][1][1] - v[0][1][0]) * tx;
    double x01 = v[1][0][0] + (v[1][0][1] - v[1][0][0]) * tx;
    double x11 = v[1][1][0] + (v[1][1][1] - v[1][1][0]) * tx;
    double y0 = x00 + (x10 - x00) * ty;
    double y1 = x01 + (x11 - x01) * ty;
    return y0 + (y1 - y0) * tz;
}

static double fbm(uint32_t seed, double x, double y, double z) {
    double sum = 0.0, norm = 0.0, amp = 1.0, freq = 4.0;
    for (int o = 0; o < 4; ++o) {
        sum += amp * value_noise(seed, o, x * freq, y * freq, z * freq);
        norm += amp;
        amp *= 0.5;
        freq *= 2.0;
    }
    return sum / norm;
}

typedef struct {
    int R;
    float* sigma;   /* R^3, x fastest */
    float* albedo;  /* R^3 or NULL (constant) */
    double albedo_const;
    double majorant;
} medium;

static int build_medium(const sg_config* c, medium* m) {
    int R = c->R;
    size_t n = (size_t)R * R * R;
    m->R = R;
    m->sigma = (float*)malloc(n * sizeof(float));
    m->albedo = NULL;
    m->albedo_const = c->albedo_lo;
    if (!m->sigma) return -1;
    if (c->albedo_mode == 1) {
        m->albedo = (float*)malloc(n * sizeof(float));
        if (!m->albedo) return -1;
    }
    uint32_t dseed = (uint32_t)splitmix64(c->seed);
    uint32_t aseed = (uint32_t)splitmix64(c->seed ^ 0xA1BED0ULL);
    double vmax = 0.0;
    #pragma omp parallel for schedule(static) reduction(max:vmax)
    for (int iz = 0; iz < R; ++iz) {
        for (int iy = 0; iy < R; ++iy) {
            for (int ix = 0; ix < R; ++ix) {
                double x = (ix + 0.5) / R, y = (iy + 0.5) / R, z = (iz + 0.5) / R;
                double n = 0.5 + c->density_contrast * (fbm(dseed, x, y, z) - 0.5) + c->density_bias;
                n = n < 0.0 ? 0.0 : (n > 1.0 ? 1.0 : n);
                double s = c->sigma_max * n;
                if (c->mask == 1) {
                    double dx = x - 0.5, dy = y - 0.5, dz = z - 0.5;
                    s *= 1.0 - smoothstep(c->mask_r0, c->mask_r1, sqrt(dx * dx + dy * dy + dz * dz));
                }
                size_t id = ((size_t)iz * R + iy) * R + ix;
                m->sigma[id] = (float)s;
                if ((double)m->sigma[id] > vmax) vmax = (double)m->sigma[id];
                if (m->albedo)
                    m->albedo[id] = (float)(c->albedo_lo + (c->albedo_hi - c->albedo_lo) *
                                    hash_unit(aseed, 7u, (uint32_t)ix, (uint32_t)iy, (uint32_t)iz));
            }
        }
    }
    m->majorant = vmax;
    return 0;
}

static size_t voxel_of(const medium* m, const double p[3]) {
    int i[3];
    for (int a = 0; a < 3; ++a) {
        int v = (int)floor(p[a] * m->R);
        i[a] = v < 0 ? 0 : (v >= m->R ? m->R - 1 : v);
    }
    return ((size_t)i[2] * m->R + i[1]) * m->R + i[0];
}
static double sigma_at(const medium* m, const double p[3]) { return m->sigma[voxel_of(m, p)]; }
static double albedo_at(const medium* m, const double p[3]) {
    return m->albedo ? (double)m->albedo[voxel_of(m, p)] : m->albedo_const;
}

/* ------------------------------------------------------------- geometry --- */
/* Ray / unit-cube slab test. Returns 1 and [t0, t1] (t0 may be < 0) on a hit. */
static int box_hit(const double o[3], const double d[3], double* t0, double* t1) {
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > 1.0) return 0;
            continue;
        }
        double inv = 1.0 / d[a];
        double ta = (0.0 - o[a]) * inv, tb = (1.0 - o[a]) * inv;
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    if (hi < lo || hi <= 0.0) return 0;
    *t0 = lo; *t1 = hi;
    return 1;
}

static void normalize3(double v[3]) {
    double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= l; v[1] /= l; v[2] /= l;
}

/* Orthonormal basis around unit n (Duff et al. 2017, "Building an orthonormal basis, revisited"). */
static void onb(const double n[3], double b1[3], double b2[3]) {
    double s = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + s * n[0] * n[0] * a; b1[1] = s * b; b1[2] = -s * n[0];
    b2[0] = b; b2[1] = s + n[1] * n[1] * a; b2[2] = -n[1];
}

/* Sample a direction whose cosine with the travel direction t follows HG(g). */
static void sample_hg(const double t[3], double g, double u1, double u2, double w[3]) {
    double mu;
    if (fabs(g) < 1e-3) {
        mu = 1.0 - 2.0 * u1;
    } else {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u1);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = 2.0 * M_PI * u2;
    double b1[3], b2[3];
    onb(t, b1, b2);
    for (int a = 0; a < 3; ++a) w[a] = mu * t[a] + st * (cos(phi) * b1[a] + sin(phi) * b2[a]);
    normalize3(w);
}

static void sample_sphere(double u1, double u2, double w[3]) {
    double z = 1.0 - 2.0 * u1;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    double phi = 2.0 * M_PI * u2;
    w[0] = r * cos(phi); w[1] = r * sin(phi); w[2] = z;
    normalize3(w);
}

/* Analog delta tracking on [t0, t1) from o along d.  Returns 1 and the
 * collision point in p on a real collision, 0 on escape. */
static int delta_track(const medium* m, pcg32* rng, const double o[3], const double d[3],
                       double t0, double t1, double p[3]) {
    if (m->majorant <= 0.0) return 0;
    double t = t0;
    for (;;) {
        t -= log(1.0 - rnd(rng)) / m->majorant;
        if (t >= t1) return 0;
        for (int a = 0; a < 3; ++a) p[a] = o[a] + t * d[a];
        if (rnd(rng) * m->majorant < sigma_at(m, p)) return 1;
    }
}

/* Ratio-tracking transmittance estimate on [0, t1) from o along d. */
static double ratio_track(const medium* m, pcg32* rng, const double o[3], const double d[3], double t1) {
    if (m->majorant <= 0.0) return 1.0;
    double T = 1.0, t = 0.0, p[3];
    for (;;) {
        t -= log(1.0 - rnd(rng)) / m->majorant;
        if (t >= t1) return T;
        for (int a = 0; a < 3; ++a) p[a] = o[a] + t * d[a];
        T *= 1.0 - sigma_at(m, p) / m->majorant;
        if (T == 0.0) return 0.0;
    }
}

static double exit_distance(const double o[3], const double d[3]) {
    double t0, t1;
    if (!box_hit(o, d, &t0, &t1)) return 0.0;
    return t1 > 0.0 ? t1 : 0.0;
}

/* ---------------------------------------------------------------- paths --- */
enum { REC = 28 }; /* floats per vertex record: pos3 din3 dout3 alb1 ls3 denv3 le3 lp3 dpl3 lpl3 */

typedef struct {
    int64_t np;       /* paths in this block */
    int64_t nv, cap;  /* vertices */
    float* rec;       /* nv * REC */
    int32_t* count;   /* np */
    float* ecam;      /* np * 3 */
    float* extra;     /* np * M * 9: (sun, env direction, env radiance) per extra sample, or NULL */
} block;

typedef struct {
    sg_config cfg;
    medium med;
    int64_t n_paths, n_vertices;
    int64_t nblocks, paths_per_block;
    block* blocks;
} handle;

static int push_vertex(block* b, const float* r) {
    if (b->nv == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        float* nr = (float*)realloc(b->rec, (size_t)nc * REC * sizeof(float));
        if (!nr) return -1;
        b->rec = nr;
        b->cap = nc;
    }
    memcpy(b->rec + (size_t)b->nv * REC, r, REC * sizeof(float));
    b->nv++;
    return 0;
}

static void camera_ray(const sg_config* c, int X, int Y, double u1, double u2, double d[3]) {
    double f[3], r[3], up[3], wup[3] = {0.0, 1.0, 0.0};
    for (int a = 0; a < 3; ++a) f[a] = c->look_at[a] - c->cam_pos[a];
    normalize3(f);
    r[0] = f[1] * wup[2] - f[2] * wup[1];
    r[1] = f[2] * wup[0] - f[0] * wup[2];
    r[2] = f[0] * wup[1] - f[1] * wup[0];
    normalize3(r);
    up[0] = r[1] * f[2] - r[2] * f[1];
    up[1] = r[2] * f[0] - r[0] * f[2];
    up[2] = r[0] * f[1] - r[1] * f[0];
    double th = tan(0.5 * c->vfov_deg * M_PI / 180.0);
    double aspect = (double)c->width / (double)c->height;
    double sx = ((X + u1) / c->width * 2.0 - 1.0) * th * aspect;
    double sy = (1.0 - (Y + u2) / c->height * 2.0) * th;
    for (int a = 0; a < 3; ++a) d[a] = f[a] + sx * r[a] + sy * up[a];
    normalize3(d);
}

/* Extra emitter samples at a path's first vertex p (paper, "Handling direct
 * Light"): M pairs of a sun shadow ray and a uniform-sphere environment
 * shadow ray, from their own PCG32 stream (the path's stream is untouched,
 * so the paths do not depend on M).  Writes M * 9 floats. */
static void extra_samples(const handle* h, uint64_t pixel, int s, const double p[3], float* out) {
    const sg_config* c = &h->cfg;
    const medium* m = &h->med;
    pcg32 rng;
    pcg32_seed(&rng, splitmix64(c->seed * 0x100000001B3ULL + (uint64_t)s) ^ 0x5851F42D4C957F2DULL, pixel);
    for (int k = 0; k < c->extra_samples; ++k) {
        float* o = out + (size_t)k * 9;
        double Ts = ratio_track(m, &rng, p, c->sun_dir, exit_distance(p, c->sun_dir));
        double v2 = rnd(&rng), v1 = rnd(&rng);
        double we[3];
        sample_sphere(v1, v2, we);
        double Te = ratio_track(m, &rng, p, we, exit_distance(p, we));
        for (int a = 0; a < 3; ++a) {
            o[a] = (float)(c->sun_E[a] * Ts);
            o[3 + a] = (float)we[a];
            o[6 + a] = (float)(c->env_L[a] * Te);
        }
    }
}

/* Trace one path; appends its vertices to b and returns the vertex count (or -1).
 * extra (M * 9 floats, zero-filled by the caller) receives the first vertex's
 * extra emitter samples. */
static int trace_path(const handle* h, block* b, int X, int Y, int s, float ecam[3], float* extra) {
    const sg_config* c = &h->cfg;
    const medium* m = &h->med;
    pcg32 rng;
    uint64_t pixel = (uint64_t)Y * (uint64_t)c->width + (uint64_t)X;
    pcg32_seed(&rng, splitmix64(c->seed * 0x100000001B3ULL + (uint64_t)s), pixel);

    double d[3], o[3], p[3], t0, t1;
    /* the pixel jitter takes the stream's first two numbers, y-jitter first */
    double jy = rnd(&rng), jx = rnd(&rng);
    camera_ray(c, X, Y, jx, jy, d);
    for (int a = 0; a < 3; ++a) o[a] = c->cam_pos[a];
    ecam[0] = ecam[1] = ecam[2] = 0.0f;
    if (!box_hit(o, d, &t0, &t1) || !delta_track(m, &rng, o, d, fmax(t0, 0.0), t1, p)) {
        for (int a = 0; a < 3; ++a) ecam[a] = (float)c->env_L[a];
        return 0;
    }
    if (extra && c->extra_samples > 0) extra_samples(h, pixel, s, p, extra);
    int nv = 0;
    for (int depth = 0; depth < c->max_depth; ++depth) {
        float r[REC];
        double we[3], wo[3], q[3];
        for (int a = 0; a < 3; ++a) { r[0 + a] = (float)p[a]; r[3 + a] = (float)d[a]; }
        r[9] = (float)albedo_at(m, p);
        /* sun shadow ray (delta light) */
        double Ts = ratio_track(m, &rng, p, c->sun_dir, exit_distance(p, c->sun_dir));
        for (int a = 0; a < 3; ++a) r[10 + a] = (float)(c->sun_E[a] * Ts);
        /* environment shadow ray, uniform sphere (azimuth number drawn first) */
        double v2 = rnd(&rng), v1 = rnd(&rng);
        sample_sphere(v1, v2, we);
        double Te = ratio_track(m, &rng, p, we, exit_distance(p, we));
        for (int a = 0; a < 3; ++a) { r[13 + a] = (float)we[a]; r[16 + a] = (float)(c->env_L[a] * Te); }
        /* point light shadow ray (delta light): irradiance I T / r^2 */
        for (int a = 0; a < 6; ++a) r[22 + a] = 0.0f;
        if (c->point_light) {
            double dl[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) { dl[a] = c->pl_pos[a] - p[a]; r2 += dl[a] * dl[a]; }
            double dist = sqrt(r2);
            for (int a = 0; a < 3; ++a) dl[a] /= dist;
            double tmax = exit_distance(p, dl);
            if (dist < tmax) tmax = dist;
            double Tp = ratio_track(m, &rng, p, dl, tmax);
            for (int a = 0; a < 3; ++a) { r[22 + a] = (float)dl[a]; r[25 + a] = (float)(c->pl_I[a] * Tp / r2); }
        }
        /* phase-sampled continuation (azimuth number drawn first) */
        double h2 = rnd(&rng), h1 = rnd(&rng);
        sample_hg(d, c->g, h1, h2, wo);
        for (int a = 0; a < 3; ++a) r[6 + a] = (float)wo[a];
        int last = (depth == c->max_depth - 1);
        int escaped = 0;
        if (!last) {
            double te = exit_distance(p, wo);
            if (!delta_track(m, &rng, p, wo, 0.0, te, q)) escaped = 1;
        }
        for (int a = 0; a < 3; ++a) r[19 + a] = escaped ? (float)c->env_L[a] : 0.0f;
        if (push_vertex(b, r)) return -1;
        ++nv;
        if (last || escaped) break;
        for (int a = 0; a < 3; ++a) { p[a] = q[a]; d[a] = wo[a]; }
    }
    return nv;
}

/* One-entry cache of the last medium built, keyed by the settings that
 * define it, so a probe render and the full render of one scene build the
 * density grid once.  Calls are not concurrent (the Python side serialises). */
static sg_config g_cached_cfg;
static medium g_cached_med;
static int g_cached_valid = 0;

static int same_medium(const sg_config* a, const sg_config* b) {
    return a->R == b->R && a->mask == b->mask && a->albedo_mode == b->albedo_mode && a->sigma_max == b->sigma_max &&
           a->density_contrast == b->density_contrast && a->density_bias == b->density_bias &&
           a->mask_r0 == b->mask_r0 && a->mask_r1 == b->mask_r1 && a->albedo_lo == b->albedo_lo &&
           a->albedo_hi == b->albedo_hi && a->seed == b->seed;
}

static int get_medium(const sg_config* c, medium* m) {
    if (!(g_cached_valid && same_medium(c, &g_cached_cfg))) {
        if (g_cached_valid) {
            free(g_cached_med.sigma);
            free(g_cached_med.albedo);
            g_cached_valid = 0;
        }
        memset(&g_cached_med, 0, sizeof g_cached_med);
        if (build_medium(c, &g_cached_med)) {
            free(g_cached_med.sigma);
            free(g_cached_med.albedo);
            return -1;
        }
        g_cached_cfg = *c;
        g_cached_valid = 1;
    }
    *m = g_cached_med;   /* shared, read-only; never freed with the handle */
    return 0;
}

static void free_handle(handle* h) {
    if (!h) return;
    if (h->blocks) {
        for (int64_t i = 0; i < h->nblocks; ++i) {
            free(h->blocks[i].rec);
            free(h->blocks[i].count);
            free(h->blocks[i].ecam);
            free(h->blocks[i].extra);
        }
        free(h->blocks);
    }
    free(h);
}

/* Trace every path of the (cropped) image.  Returns an opaque handle and the
 * vertex / path counts, or NULL (message in err). */
void* sg_trace(const sg_config* cfg, int nthreads, int64_t* n_vertices, int64_t* n_paths,
               char* err, int errlen) {
    if (cfg->R < 1 || cfg->width < 1 || cfg->height < 1 || cfg->spp < 1 || cfg->max_depth < 1 ||
        cfg->sigma_max < 0.0 || fabs(cfg->g) >= 1.0 || cfg->extra_samples < 0 || cfg->extra_samples > 1024) {
        snprintf(err, errlen, "invalid scene configuration");
        return NULL;
    }
    int cw = cfg->crop_w ? cfg->crop_w : cfg->width;
    int ch = cfg->crop_w ? cfg->crop_h : cfg->height;
    int cx0 = cfg->crop_w ? cfg->crop_x0 : 0, cy0 = cfg->crop_w ? cfg->crop_y0 : 0;
    if (cw < 1 || ch < 1 || cx0 < 0 || cy0 < 0 || cx0 + cw > cfg->width || cy0 + ch > cfg->height) {
        snprintf(err, errlen, "invalid crop window");
        return NULL;
    }
    handle* h = (handle*)calloc(1, sizeof(handle));
    if (!h) { snprintf(err, errlen, "out of memory"); return NULL; }
    h->cfg = *cfg;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (get_medium(cfg, &h->med)) { snprintf(err, errlen, "out of memory"); free_handle(h); return NULL; }
    h->n_paths = (int64_t)cw * ch * cfg->spp;
    h->paths_per_block = 256;
    h->nblocks = (h->n_paths + h->paths_per_block - 1) / h->paths_per_block;
    h->blocks = (block*)calloc((size_t)h->nblocks, sizeof(block));
    if (!h->blocks) { snprintf(err, errlen, "out of memory"); free_handle(h); return NULL; }
    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t bi = 0; bi < h->nblocks; ++bi) {
        block* b = &h->blocks[bi];
        int64_t p0 = bi * h->paths_per_block;
        int64_t p1 = p0 + h->paths_per_block;
        if (p1 > h->n_paths) p1 = h->n_paths;
        b->np = p1 - p0;
        b->count = (int32_t*)malloc((size_t)b->np * sizeof(int32_t));
        b->ecam = (float*)malloc((size_t)b->np * 3 * sizeof(float));
        const size_t M9 = (size_t)cfg->extra_samples * 9;
        b->extra = M9 ? (float*)calloc((size_t)b->np * M9, sizeof(float)) : NULL;
        if (!b->count || !b->ecam || (M9 && !b->extra)) { fail = 1; continue; }
        for (int64_t p = p0; p < p1; ++p) {
            int64_t pix = p / cfg->spp;
            int s = (int)(p % cfg->spp);
            int X = cx0 + (int)(pix % cw), Y = cy0 + (int)(pix / cw);
            int nv = trace_path(h, b, X, Y, s, b->ecam + (p - p0) * 3, M9 ? b->extra + (p - p0) * M9 : NULL);
            if (nv < 0) { fail = 1; break; }
            b->count[p - p0] = nv;
        }
    }
    if (fail) { snprintf(err, errlen, "out of memory while tracing"); free_handle(h); return NULL; }
    int64_t nv = 0;
    for (int64_t bi = 0; bi < h->nblocks; ++bi) nv += h->blocks[bi].nv;
    h->n_vertices = nv;
    *n_vertices = nv;
    *n_paths = h->n_paths;
    return h;
}

/* Copy the traced records, in path order, into caller arrays
 * (path_offsets[P+1], per-vertex [N][3] or [N], e_cam[P][3]). */
int sg_fetch(void* hp, int64_t* path_offsets, float* pos, float* dir_in, float* dir_out,
             float* albedo, float* l_sun, float* dir_env, float* l_env, float* l_phase, float* e_cam) {
    handle* h = (handle*)hp;
    int64_t* vstart = (int64_t*)malloc((size_t)(h->nblocks + 1) * sizeof(int64_t));
    if (!vstart) return -1;
    vstart[0] = 0;
    for (int64_t bi = 0; bi < h->nblocks; ++bi) vstart[bi + 1] = vstart[bi] + h->blocks[bi].nv;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t bi = 0; bi < h->nblocks; ++bi) {
        const block* b = &h->blocks[bi];
        int64_t p0 = bi * h->paths_per_block;
        int64_t off = vstart[bi];
        for (int64_t i = 0; i < b->np; ++i) {
            path_offsets[p0 + i] = off;
            off += b->count[i];
            for (int a = 0; a < 3; ++a) e_cam[(p0 + i) * 3 + a] = b->ecam[i * 3 + a];
        }
        for (int64_t v = 0; v < b->nv; ++v) {
            const float* r = b->rec + (size_t)v * REC;
            int64_t gv = vstart[bi] + v;
            for (int a = 0; a < 3; ++a) {
                pos[gv * 3 + a] = r[0 + a];
                dir_in[gv * 3 + a] = r[3 + a];
                dir_out[gv * 3 + a] = r[6 + a];
                l_sun[gv * 3 + a] = r[10 + a];
                dir_env[gv * 3 + a] = r[13 + a];
                l_env[gv * 3 + a] = r[16 + a];
                l_phase[gv * 3 + a] = r[19 + a];
            }
            albedo[gv] = r[9];
        }
    }
    path_offsets[h->n_paths] = vstart[h->nblocks];
    free(vstart);
    return 0;
}

/* Copy the density grid (R^3 floats, x fastest) and return the majorant. */
double sg_density(void* hp, float* sigma_out) {
    handle* h = (handle*)hp;
    size_t n = (size_t)h->med.R * h->med.R * h->med.R;
    memcpy(sigma_out, h->med.sigma, n * sizeof(float));
    return h->med.majorant;
}

/* Copy the point-light records (direction, irradiance x transmittance),
 * [N][3] each, path order; 1 if the scene has no point light. */
int sg_fetch_point_light(void* hp, float* dir_pl, float* l_pl) {
    handle* h = (handle*)hp;
    if (!h->cfg.point_light) return 1;
    int64_t* vstart = (int64_t*)malloc((size_t)(h->nblocks + 1) * sizeof(int64_t));
    if (!vstart) return -1;
    vstart[0] = 0;
    for (int64_t bi = 0; bi < h->nblocks; ++bi) vstart[bi + 1] = vstart[bi] + h->blocks[bi].nv;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t bi = 0; bi < h->nblocks; ++bi) {
        const block* b = &h->blocks[bi];
        for (int64_t v = 0; v < b->nv; ++v) {
            const float* r = b->rec + (size_t)v * REC;
            int64_t gv = vstart[bi] + v;
            for (int a = 0; a < 3; ++a) {
                dir_pl[gv * 3 + a] = r[22 + a];
                l_pl[gv * 3 + a] = r[25 + a];
            }
        }
    }
    free(vstart);
    return 0;
}

/* Copy the extra first-vertex emitter samples, [P][M] each of l_sun[3],
 * dir_env[3], l_env[3] (zero for a path without vertices); 1 if M == 0. */
int sg_fetch_extra(void* hp, float* fb_l_sun, float* fb_dir_env, float* fb_l_env) {
    handle* h = (handle*)hp;
    const int64_t M = h->cfg.extra_samples;
    if (M == 0) return 1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t bi = 0; bi < h->nblocks; ++bi) {
        const block* b = &h->blocks[bi];
        int64_t p0 = bi * h->paths_per_block;
        for (int64_t i = 0; i < b->np; ++i)
            for (int64_t k = 0; k < M; ++k) {
                const float* e = b->extra + ((size_t)i * M + k) * 9;
                const size_t o = ((size_t)(p0 + i) * M + k) * 3;
                for (int a = 0; a < 3; ++a) {
                    fb_l_sun[o + a] = e[a];
                    fb_dir_env[o + a] = e[3 + a];
                    fb_l_env[o + a] = e[6 + a];
                }
            }
    }
    return 0;
}

/* Copy the per-voxel albedo grid (R^3 floats, x fastest); 1 if the albedo is constant. */
int sg_albedo(void* hp, float* albedo_out) {
    handle* h = (handle*)hp;
    if (!h->med.albedo) return 1;
    size_t n = (size_t)h->med.R * h->med.R * h->med.R;
    memcpy(albedo_out, h->med.albedo, n * sizeof(float));
    return 0;
}

void sg_release(void* hp) { free_handle((handle*)hp); }
