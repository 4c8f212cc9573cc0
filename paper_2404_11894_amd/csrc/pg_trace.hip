// pg_trace.hip -- the instrumented delta-tracking volume path tracer on the
// GPU: the upstream step that produces the path-ordered vertex records (paper
// Sec. "Volume Path Tracing"; Sec. "Rendering System", instrumented path
// tracer: per shading point the emitter-sampling and phase-sampling data and
// the radiance of its continuation), written straight into HBM.
//
// Medium: a grid of extinction coefficients over the unit cube (nearest
// voxel, x fastest), vacuum outside; albedo per voxel or constant.  Lights:
// a directional (delta) sun and a constant environment.  Per path: a camera
// ray through the pixel (jittered), analog delta tracking against the grid
// majorant; at every real collision a sun shadow ray and one uniform-sphere
// environment shadow ray, both with ratio-tracking transmittance, and a
// continuation sampled from Henyey-Greenstein about the arriving direction;
// at most max_depth vertices, the last without continuation; no Russian
// roulette.  Random numbers: PCG32 (O'Neill 2014), one stream per pixel of
// the full image, seeded from (seed, sample index) through splitmix64, so a
// crop traces the paths the full image traces there.
//
// One thread per path, in double precision without contraction.  The
// counting pass traces each path into max_depth record slots of its own in
// the workspace; a scan gives the offsets, and the record pass copies each
// path's records to its offsets.
#include <cmath>

#include "pg_api_common.h"

#pragma clang fp contract(off)

namespace pg {

namespace {

struct Rng {
    uint64_t state, inc;
    __device__ uint32_t next() {
        const uint64_t old = state;
        state = old * 6364136223846793005ull + inc;
        const uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
        const uint32_t rot = (uint32_t)(old >> 59u);
        return (xs >> rot) | (xs << ((0u - rot) & 31u));
    }
    __device__ void seed(uint64_t initstate, uint64_t initseq) {
        state = 0u;
        inc = (initseq << 1u) | 1u;
        (void)next();
        state += initstate;
        (void)next();
    }
    __device__ double uniform() { return (double)next() * (1.0 / 4294967296.0); }   // [0, 1), 32 bits
};

__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

struct D3 {
    double x, y, z;
};
__device__ inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ inline double comp(const D3& v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

__device__ inline D3 normalized(D3 v) {
    const double l = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    return d3(v.x / l, v.y / l, v.z / l);
}

struct Tracer {
    pg_tracer t;
    int cw, ch, cx0, cy0;
    int point_light;
    // camera frame
    D3 f, r, up;
    double th, aspect;
};

__device__ inline size_t voxel_of(const pg_tracer& t, const D3& p) {
    int i[3];
    for (int a = 0; a < 3; ++a) {
        const int v = (int)floor(comp(p, a) * t.R);
        i[a] = v < 0 ? 0 : (v >= t.R ? t.R - 1 : v);
    }
    return ((size_t)i[2] * t.R + i[1]) * t.R + i[0];
}

__device__ inline double sigma_at(const pg_tracer& t, const D3& p) { return (double)t.sigma[voxel_of(t, p)]; }

__device__ inline double albedo_at(const pg_tracer& t, const D3& p) {
    return t.albedo ? (double)t.albedo[voxel_of(t, p)] : t.albedo_const;
}

// Ray / unit-cube slab test: 1 and [t0, t1] (t0 may be < 0) on a hit.
__device__ inline int box_hit(const D3& o, const D3& d, double& t0, double& t1) {
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double oa = comp(o, a), da = comp(d, a);
        if (da == 0.0) {
            if (oa < 0.0 || oa > 1.0) return 0;
            continue;
        }
        const double inv = 1.0 / da;
        double ta = (0.0 - oa) * inv, tb = (1.0 - oa) * inv;
        if (ta > tb) {
            const double tt = ta;
            ta = tb;
            tb = tt;
        }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    if (hi < lo || hi <= 0.0) return 0;
    t0 = lo;
    t1 = hi;
    return 1;
}

__device__ inline double exit_distance(const D3& o, const D3& d) {
    double t0, t1;
    if (!box_hit(o, d, t0, t1)) return 0.0;
    return t1 > 0.0 ? t1 : 0.0;
}

// Orthonormal basis around unit n (Duff et al. 2017).
__device__ inline void onb(const D3& n, D3& b1, D3& b2) {
    const double s = n.z >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (s + n.z);
    const double b = n.x * n.y * a;
    b1 = d3(1.0 + s * n.x * n.x * a, s * b, -s * n.x);
    b2 = d3(b, s + n.y * n.y * a, -n.y);
}

// Direction whose cosine with the travel direction t follows HG(g) (inversion).
__device__ inline D3 sample_hg(const D3& t, double g, double u1, double u2) {
    double mu;
    if (fabs(g) < 1e-3) {
        mu = 1.0 - 2.0 * u1;
    } else {
        const double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u1);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    const double phi = 2.0 * M_PI * u2;
    D3 b1, b2;
    onb(t, b1, b2);
    const double c = cos(phi), sn = sin(phi);
    return normalized(d3(mu * t.x + st * (c * b1.x + sn * b2.x), mu * t.y + st * (c * b1.y + sn * b2.y),
                         mu * t.z + st * (c * b1.z + sn * b2.z)));
}

__device__ inline D3 sample_sphere(double u1, double u2) {
    const double z = 1.0 - 2.0 * u1;
    const double r = sqrt(fmax(0.0, 1.0 - z * z));
    const double phi = 2.0 * M_PI * u2;
    return normalized(d3(r * cos(phi), r * sin(phi), z));
}

// Analog delta tracking on [t0, t1): 1 and the collision point on a real collision.
__device__ inline int delta_track(const pg_tracer& t, Rng& rng, const D3& o, const D3& d, double t0, double t1,
                                  D3& p) {
    const double maj = t.majorant;
    if (maj <= 0.0) return 0;
    double s = t0;
    for (;;) {
        s -= log(1.0 - rng.uniform()) / maj;
        if (s >= t1) return 0;
        p = d3(o.x + s * d.x, o.y + s * d.y, o.z + s * d.z);
        if (rng.uniform() * maj < sigma_at(t, p)) return 1;
    }
}

// Ratio-tracking transmittance estimate on [0, t1).
__device__ inline double ratio_track(const pg_tracer& t, Rng& rng, const D3& o, const D3& d, double t1) {
    const double maj = t.majorant;
    if (maj <= 0.0) return 1.0;
    double T = 1.0, s = 0.0;
    for (;;) {
        s -= log(1.0 - rng.uniform()) / maj;
        if (s >= t1) return T;
        const D3 p = d3(o.x + s * d.x, o.y + s * d.y, o.z + s * d.z);
        T *= 1.0 - sigma_at(t, p) / maj;
        if (T == 0.0) return 0.0;
    }
}

struct Out {
    float *pos, *dir_in, *dir_out, *albedo, *l_sun, *dir_env, *l_env, *l_phase;
    float *fb_l_sun, *fb_dir_env, *fb_l_env;   // [P][M][3]
    float *dir_pl, *l_pl;
};

// The M extra emitter samples at a path's first vertex pt (paper, handling
// direct light): sun and uniform-sphere environment shadow rays from a
// second stream of the pixel, so the path itself does not depend on M.
__device__ void extra_samples(const pg_tracer& t, uint64_t pixel, int s, const D3& pt, int64_t p, const Out& o) {
    Rng rng;
    rng.seed(splitmix64(t.seed * 0x100000001B3ull + (uint64_t)s) ^ 0x5851F42D4C957F2Dull, pixel);
    const D3 sun = d3(t.sun_dir[0], t.sun_dir[1], t.sun_dir[2]);
    for (int k = 0; k < t.extra_samples; ++k) {
        const double Ts = ratio_track(t, rng, pt, sun, exit_distance(pt, sun));
        const double v2 = rng.uniform();   // azimuth number first
        const double v1 = rng.uniform();
        const D3 we = sample_sphere(v1, v2);
        const double Te = ratio_track(t, rng, pt, we, exit_distance(pt, we));
        const int64_t b = ((int64_t)p * t.extra_samples + k) * 3;
        for (int a = 0; a < 3; ++a) {
            o.fb_l_sun[b + a] = (float)(t.sun_E[a] * Ts);
            o.fb_dir_env[b + a] = (float)comp(we, a);
            o.fb_l_env[b + a] = (float)(t.env_L[a] * Te);
        }
    }
}

// Traces path p of the (cropped) image; with WRITE stores its records from
// slot v0 on.  Returns the vertex count; ecam receives the camera ray's
// environment radiance when it escapes.
template <bool WRITE>
__device__ int trace_path(const Tracer& tr, int64_t p, int64_t v0, int64_t vcap, const Out& o, float ecam[3]) {
    const pg_tracer& t = tr.t;
    const int64_t pix = p / t.spp;
    const int s = (int)(p % t.spp);
    const int X = tr.cx0 + (int)(pix % tr.cw), Y = tr.cy0 + (int)(pix / tr.cw);
    Rng rng;
    rng.seed(splitmix64(t.seed * 0x100000001B3ull + (uint64_t)s), (uint64_t)Y * (uint64_t)t.width + (uint64_t)X);
    const double u2 = rng.uniform();   // the jitter: y first, then x
    const double u1 = rng.uniform();
    const double sx = ((X + u1) / t.width * 2.0 - 1.0) * tr.th * tr.aspect;
    const double sy = (1.0 - (Y + u2) / t.height * 2.0) * tr.th;
    D3 d = normalized(d3(tr.f.x + sx * tr.r.x + sy * tr.up.x, tr.f.y + sx * tr.r.y + sy * tr.up.y,
                         tr.f.z + sx * tr.r.z + sy * tr.up.z));
    const D3 cam = d3(t.cam_pos[0], t.cam_pos[1], t.cam_pos[2]);
    ecam[0] = ecam[1] = ecam[2] = 0.0f;
    double t0, t1;
    D3 pt;
    if (!box_hit(cam, d, t0, t1) || !delta_track(t, rng, cam, d, fmax(t0, 0.0), t1, pt)) {
        for (int a = 0; a < 3; ++a) ecam[a] = (float)t.env_L[a];
        if (WRITE && t.extra_samples > 0)   // no first vertex: zero samples
            for (int64_t b = p * t.extra_samples * 3; b < (p + 1) * t.extra_samples * 3; ++b)
                o.fb_l_sun[b] = o.fb_dir_env[b] = o.fb_l_env[b] = 0.0f;
        return 0;
    }
    if (WRITE && t.extra_samples > 0)
        extra_samples(t, (uint64_t)Y * (uint64_t)t.width + (uint64_t)X, s, pt, p, o);
    const D3 sun = d3(t.sun_dir[0], t.sun_dir[1], t.sun_dir[2]);
    int nv = 0;
    for (int depth = 0; depth < t.max_depth; ++depth) {
        const double alb = albedo_at(t, pt);
        const double Ts = ratio_track(t, rng, pt, sun, exit_distance(pt, sun));
        const double e2 = rng.uniform();   // azimuth number first
        const double e1 = rng.uniform();
        const D3 we = sample_sphere(e1, e2);
        const double Te = ratio_track(t, rng, pt, we, exit_distance(pt, we));
        // point light shadow ray (delta light): irradiance I T / r^2
        D3 dl = d3(0.0, 0.0, 0.0);
        double lpl[3] = {0.0, 0.0, 0.0};
        bool pl_zero = true;
        if (tr.point_light) {
            D3 v = d3(t.pl_pos[0] - pt.x, t.pl_pos[1] - pt.y, t.pl_pos[2] - pt.z);
            const double r2 = v.x * v.x + v.y * v.y + v.z * v.z;
            const double dist = sqrt(r2);
            dl = d3(v.x / dist, v.y / dist, v.z / dist);
            double tmax = exit_distance(pt, dl);
            if (dist < tmax) tmax = dist;
            const double Tp = ratio_track(t, rng, pt, dl, tmax);
            for (int a = 0; a < 3; ++a) lpl[a] = t.pl_I[a] * Tp / r2;
            pl_zero = false;
        }
        const double h2 = rng.uniform();   // azimuth number first
        const double h1 = rng.uniform();
        const D3 wo = sample_hg(d, t.g, h1, h2);
        const bool last = depth == t.max_depth - 1;
        bool escaped = false;
        D3 q = pt;
        if (!last) {
            const double te = exit_distance(pt, wo);
            if (!delta_track(t, rng, pt, wo, 0.0, te, q)) escaped = true;
        }
        if (WRITE && nv < vcap) {   // never past the path's slots
            const int64_t v = v0 + nv;
            for (int a = 0; a < 3; ++a) {
                o.pos[3 * v + a] = (float)comp(pt, a);
                o.dir_in[3 * v + a] = (float)comp(d, a);
                o.dir_out[3 * v + a] = (float)comp(wo, a);
                o.l_sun[3 * v + a] = (float)(t.sun_E[a] * Ts);
                o.dir_env[3 * v + a] = (float)comp(we, a);
                o.l_env[3 * v + a] = (float)(t.env_L[a] * Te);
                o.l_phase[3 * v + a] = escaped ? (float)t.env_L[a] : 0.0f;
            }
            o.albedo[v] = (float)alb;
            if (tr.point_light)
                for (int a = 0; a < 3; ++a) {
                    o.dir_pl[3 * v + a] = pl_zero ? 0.0f : (float)comp(dl, a);
                    o.l_pl[3 * v + a] = (float)lpl[a];
                }
        }
        ++nv;
        if (last || escaped) break;
        pt = q;
        d = wo;
    }
    return nv;
}

// Pass 1: traces path p into its max_depth slots of the workspace slab
// (slot p * max_depth + k), with its extra samples and camera term, and
// counts its vertices.
__global__ __launch_bounds__(kBlock) void k_trace_count(Tracer tr, int64_t P, uint32_t* __restrict__ count, Out slab,
                                                        float* __restrict__ slab_ecam) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float ec[3];
    const int64_t maxd = tr.t.max_depth;
    count[p] = (uint32_t)trace_path<true>(tr, p, p * maxd, maxd, slab, ec);
    for (int a = 0; a < 3; ++a) slab_ecam[3 * p + a] = ec[a];
}

// Pass 2: one thread per slab slot (p, k) copies the k-th record of path p
// to path_offsets[p] + k.  A path whose offsets do not span exactly its
// traced vertex count (offsets not from this trace) is not written and is
// reported.
__global__ __launch_bounds__(kBlock) void k_trace_compact(int64_t P, int64_t maxd, const int64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ start, Out slab, Out o,
                                                          bool point_light, int32_t* flag) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= P * maxd) return;
    const int64_t p = slot / maxd, k = slot - p * maxd;
    const int64_t c = (int64_t)start[p + 1] - (int64_t)start[p];
    const int64_t a = off[p], n = off[p + 1] - a;
    if (n != c || a < 0) {
        if (k == 0) set_flag(flag, kFlagOffsets);   // offsets not from this tracer
        return;
    }
    if (k >= c) return;
    const int64_t v = a + k;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o.pos[3 * v + q] = slab.pos[3 * slot + q];
        o.dir_in[3 * v + q] = slab.dir_in[3 * slot + q];
        o.dir_out[3 * v + q] = slab.dir_out[3 * slot + q];
        o.l_sun[3 * v + q] = slab.l_sun[3 * slot + q];
        o.dir_env[3 * v + q] = slab.dir_env[3 * slot + q];
        o.l_env[3 * v + q] = slab.l_env[3 * slot + q];
        o.l_phase[3 * v + q] = slab.l_phase[3 * slot + q];
        if (point_light) {
            o.dir_pl[3 * v + q] = slab.dir_pl[3 * slot + q];
            o.l_pl[3 * v + q] = slab.l_pl[3 * slot + q];
        }
    }
    o.albedo[v] = slab.albedo[slot];
}

// offsets (int64) from the scanned counts (uint32, P+1 entries)
__global__ __launch_bounds__(kBlock) void k_widen(int64_t n, const uint32_t* __restrict__ in, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace

static Tracer make_tracer(const pg_tracer* t) {
    Tracer tr;
    tr.t = *t;
    tr.cw = t->crop_w ? t->crop_w : t->width;
    tr.ch = t->crop_w ? t->crop_h : t->height;
    tr.cx0 = t->crop_w ? t->crop_x0 : 0;
    tr.cy0 = t->crop_w ? t->crop_y0 : 0;
    tr.point_light = t->pl_I[0] != 0.0 || t->pl_I[1] != 0.0 || t->pl_I[2] != 0.0;
    // camera frame, as the device would compute it (host double, same order)
    double f[3], r[3], up[3];
    const double wup[3] = {0.0, 1.0, 0.0};
    for (int a = 0; a < 3; ++a) f[a] = t->look_at[a] - t->cam_pos[a];
    double l = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int a = 0; a < 3; ++a) f[a] /= l;
    r[0] = f[1] * wup[2] - f[2] * wup[1];
    r[1] = f[2] * wup[0] - f[0] * wup[2];
    r[2] = f[0] * wup[1] - f[1] * wup[0];
    l = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int a = 0; a < 3; ++a) r[a] /= l;
    up[0] = r[1] * f[2] - r[2] * f[1];
    up[1] = r[2] * f[0] - r[0] * f[2];
    up[2] = r[0] * f[1] - r[1] * f[0];
    tr.f = D3{f[0], f[1], f[2]};
    tr.r = D3{r[0], r[1], r[2]};
    tr.up = D3{up[0], up[1], up[2]};
    tr.th = std::tan(0.5 * t->vfov_deg * M_PI / 180.0);
    tr.aspect = (double)t->width / (double)t->height;
    return tr;
}

int64_t tracer_paths(const pg_tracer* t) {
    const int64_t cw = t->crop_w ? t->crop_w : t->width, ch = t->crop_w ? t->crop_h : t->height;
    return cw * ch * t->spp;
}

// Workspace: flags, the vertex counts (scanned in place to offsets), and the
// slab the count pass traces into: max_depth record slots per path, the
// paths' extra samples and camera terms.  Pass 2 copies from the slab, so
// both passes must use the same workspace, unchanged in between.
struct TraceWs {
    int32_t* flag;
    uint32_t* count;
    uint32_t* part;
    Out slab;
    float* ecam;
};

static TraceWs carve_trace(Carver& cv, const pg_tracer* t) {
    const int64_t P = tracer_paths(t);
    const int64_t S = P * (int64_t)t->max_depth;
    const bool pl = t->pl_I[0] != 0.0 || t->pl_I[1] != 0.0 || t->pl_I[2] != 0.0;
    const int64_t F = t->extra_samples > 0 ? P * (int64_t)t->extra_samples * 3 : 0;
    TraceWs w;
    w.flag = cv.take<int32_t>(64);
    w.count = cv.take<uint32_t>(P + 1);
    w.part = cv.take<uint32_t>(scan_partials_bytes(P + 1) / 4);
    w.slab.pos = cv.take<float>(3 * S);
    w.slab.dir_in = cv.take<float>(3 * S);
    w.slab.dir_out = cv.take<float>(3 * S);
    w.slab.albedo = cv.take<float>(S);
    w.slab.l_sun = cv.take<float>(3 * S);
    w.slab.dir_env = cv.take<float>(3 * S);
    w.slab.l_env = cv.take<float>(3 * S);
    w.slab.l_phase = cv.take<float>(3 * S);
    w.slab.fb_l_sun = F ? cv.take<float>(F) : nullptr;
    w.slab.fb_dir_env = F ? cv.take<float>(F) : nullptr;
    w.slab.fb_l_env = F ? cv.take<float>(F) : nullptr;
    w.slab.dir_pl = pl ? cv.take<float>(3 * S) : nullptr;
    w.slab.l_pl = pl ? cv.take<float>(3 * S) : nullptr;
    w.ecam = cv.take<float>(3 * P + 3);
    return w;
}

size_t trace_ws_size(const pg_tracer* t) {
    Carver cv(nullptr);
    (void)carve_trace(cv, t);
    return cv.size();
}

hipError_t run_trace_count(const pg_tracer* t, int64_t* path_offsets, float* e_cam, void* ws, hipStream_t s) {
    (void)e_cam;   // kept in the slab; pass 2 writes it
    const int64_t P = tracer_paths(t);
    Carver cv(ws);
    const TraceWs w = carve_trace(cv, t);
    hipError_t e;
    if ((e = launch_fill(w.count, (size_t)(P + 1) * 4, s)) != hipSuccess) return e;
    const Tracer tr = make_tracer(t);
    if (P > 0) {
        ProfScope ps(s, "trace_count");
        hipLaunchKernelGGL(k_trace_count, dim3((unsigned)div_up(P, kBlock)), dim3(kBlock), 0, s, tr, P, w.count,
                           w.slab, w.ecam);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_scan_exclusive(w.count, w.count, P + 1, w.part, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)div_up(P + 1, kBlock)), dim3(kBlock), 0, s, P + 1, w.count,
                       path_offsets);
    return hipGetLastError();
}

hipError_t run_trace_write(const pg_tracer* t, const int64_t* path_offsets, const pg_records& o, void* ws,
                           hipStream_t s, int32_t** flag_out) {
    const int64_t P = tracer_paths(t);
    Carver cv(ws);
    const TraceWs w = carve_trace(cv, t);
    *flag_out = w.flag;
    hipError_t e;
    if ((e = launch_fill(w.flag, 64 * 4, s)) != hipSuccess) return e;
    if (P == 0) return hipSuccess;
    const Tracer tr = make_tracer(t);
    Out out{o.pos, o.dir_in, o.dir_out, o.albedo, o.l_sun, o.dir_env, o.l_env, o.l_phase,
            o.fb_l_sun, o.fb_dir_env, o.fb_l_env, o.dir_pl, o.l_pl};
    ProfScope ps(s, "trace_write");
    const int64_t maxd = t->max_depth;
    hipLaunchKernelGGL(k_trace_compact, dim3((unsigned)div_up(P * maxd, kBlock)), dim3(kBlock), 0, s, P, maxd,
                       path_offsets, (const uint32_t*)w.count, w.slab, out, tr.point_light, w.flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(o.e_cam, w.ecam, (size_t)P * 12, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if (t->extra_samples > 0) {
        const size_t F = (size_t)P * (size_t)t->extra_samples * 12;
        if ((e = hipMemcpyAsync(o.fb_l_sun, w.slab.fb_l_sun, F, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(o.fb_dir_env, w.slab.fb_dir_env, F, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(o.fb_l_env, w.slab.fb_l_env, F, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pg
