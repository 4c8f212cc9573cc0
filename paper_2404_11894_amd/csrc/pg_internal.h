// pg_internal.h -- device helpers and launch wrappers shared by the HIP
// translation units of the path-graph library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <type_traits>

#include "../../include/pathgraph.h"

namespace pg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kQBits = 20;                    // quantisation bits per axis
constexpr uint32_t kQMax = (1u << kQBits) - 1u;
constexpr int kMinShift = 11;                 // finest grid: 2^(20-11) = 512 cells per axis
constexpr float kPi = 3.14159265358979323846f;

// Device error flags (bit mask in one int32 of the workspace).
enum : int32_t {
    kFlagPos = 1,       // non-finite or out-of-range position
    kFlagOffsets = 2,   // path offsets not monotone / out of range
    kFlagIndex = 4,     // neighbour id out of range in caller-provided CSR
    kFlagCluster = 8,   // a cluster above kClusterMax members (keys not uniform)
    kFlagCapacity = 16, // exported cluster edges exceed the caller's capacity
    kFlagRows = 32,     // caller-provided row_ptr is not the k-nearest layout i K
};

// Cluster neighbour relation: rounds of splitting large clusters, and the
// largest cluster the kernels accept (far beyond what uniform keys produce).
constexpr int kClusterRounds = 4;
constexpr int kClusterMax = 4096;

// ---------------------------------------------------------------- helpers --

__host__ __device__ inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Internal edge layout: sliced ELL with quads.  Rows are grouped in slices
// of 64 (one wave) and a row's edges in quads of four; the row stride is K
// rounded up to a multiple of 4, and the padding slots hold the row itself
// with weight 0, so a sum over all slots of the last quad adds exactly +0
// (weights and radiance are non-negative).  Inside a
// slice, quad q of all 64 rows is contiguous and each row's quad is 16 bytes,
// so a wave that owns a slice reads four edges of each of its rows with one
// 16-byte load per lane, 1 KiB contiguous per wave.
constexpr int kSlice = 64;
constexpr int64_t kQuadStride = 4 * kSlice;   // elements between quads q and q+1 of a row
__host__ __device__ inline int ell_k4(int K) { return (K + 3) & ~3; }
__host__ __device__ inline int64_t ell_row(int64_t i, int K) {   // element of edge 0 of row i
    return (i >> 6) * (int64_t)ell_k4(K) * kSlice + (i & (kSlice - 1)) * 4;
}
__host__ __device__ inline int64_t eidx(int64_t i, int l, int K) {
    return ell_row(i, K) + (l >> 2) * kQuadStride + (l & 3);
}
__host__ __device__ inline int64_t ell_size(int64_t N, int K) { return div_up(N, kSlice) * kSlice * ell_k4(K); }

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// One quad of edge ids / weights, streamed past the caches (read once).
__device__ inline i32x4 ld_quad_nt(const int32_t* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(p));
}
__device__ inline f32x4 ld_quad_nt(const float* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
}

// Workgroup b's row tile when each XCD takes G consecutive tiles in turn: the
// hardware hands workgroup b to XCD b % 8, so tiles [8Gc + Gx, 8Gc + G(x+1))
// of chunk c go to XCD x.  G = 1 is the plain launch order; the tail past the
// last whole chunk keeps plain order.  A bijection on [0, nb).
__device__ inline int64_t grouped_tile(int64_t b, int64_t nb, int G) {
    if (G <= 1) return b;
    const int64_t span = 8 * (int64_t)G;
    if (b >= (nb / span) * span) return b;
    const int64_t c = b / span, r = b - c * span;
    return c * span + (r & 7) * G + (r >> 3);
}

// Runs go(std::integral_constant<int, BS>) with the workgroup size BS of a
// propagation launch (tile 0 = 256).
template <class F>
inline void dispatch_tile(int tile, F&& go) {
    switch (tile) {
    case 64: go(std::integral_constant<int, 64>{}); break;
    case 128: go(std::integral_constant<int, 128>{}); break;
    case 512: go(std::integral_constant<int, 512>{}); break;
    case 1024: go(std::integral_constant<int, 1024>{}); break;
    default: go(std::integral_constant<int, 256>{}); break;
    }
}

// XCD-aware block order.  The hardware hands block b to XCD b % 8; remap so
// every XCD works on one contiguous range of tiles, which keeps the spatially
// sorted rows that share neighbours on the same L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, rem = nb & 7;
    const int64_t x = b & 7, k = b >> 3;
    return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

// Spread the low 10 bits of v to every third bit.
__host__ __device__ inline uint32_t part1by2(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}
// Inverse of part1by2: gather every third bit into the low 10 bits.
__host__ __device__ inline uint32_t compact1by2(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}

// Position of cell (x, y, z) along the 3-D Hilbert curve over a 2^b grid
// (b <= 10), after Skilling's transpose form of the curve (J. Skilling,
// "Programming the Hilbert curve", 2004): undo the excess work of the
// recursive rotations, Gray-encode, then interleave the bits with x most
// significant.  Consecutive positions are face-adjacent cells, unlike the
// Morton order, whose steps jump at every octant boundary.
__host__ __device__ inline uint32_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int b) {
    if (b <= 0) return 0;
    uint32_t X[3] = {x, y, z};
    const uint32_t M = 1u << (b - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    return morton3(X[2] ^ t, X[1] ^ t, X[0] ^ t);
}

// Quantised coordinates packed 21 bits apart.
__device__ inline uint64_t qpack(uint32_t x, uint32_t y, uint32_t z) {
    return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}
__device__ inline void qunpack(uint64_t p, int32_t& x, int32_t& y, int32_t& z) {
    x = (int32_t)(p & 0x1fffffu);
    y = (int32_t)((p >> 21) & 0x1fffffu);
    z = (int32_t)((p >> 42) & 0x1fffffu);
}

struct f3 { float x, y, z; };

__device__ inline f3 ld3(const float* p, int64_t i) { return f3{p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ inline void st3(float* p, int64_t i, f3 v) { p[3 * i] = v.x; p[3 * i + 1] = v.y; p[3 * i + 2] = v.z; }
// Store with the non-temporal hint: the propagation's output vectors are
// consumed by the next kernel's gathers, which measured faster when these
// stores do not allocate in the caches on the way out.
__device__ inline void st3_nt(float* p, int64_t i, f3 v) {
    __builtin_nontemporal_store(v.x, p + 3 * i);
    __builtin_nontemporal_store(v.y, p + 3 * i + 1);
    __builtin_nontemporal_store(v.z, p + 3 * i + 2);
}

// sum_l w_il x(j_l) for row i of the sliced ELL, over all K4 = ell_k4(K)
// slots (the padding slots add +0).  KT = K4 at compile time: every quad's id
// and weight load is issued before the K4 gathers, so a wave has 64*K4
// gathers in flight; KT = 0: runtime K4, quad by quad.
template <int KT>
__device__ __forceinline__ f3 ell_row_sum(int64_t i, int K, const int32_t* __restrict__ col,
                                          const float* __restrict__ w, const float* __restrict__ x) {
    static_assert(KT % 4 == 0, "compile-time K4 must fill whole quads");
    const int64_t base = ell_row(i, K);
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (KT) {
        constexpr int NQ = KT > 0 ? KT / 4 : 1;
        i32x4 j[NQ];
        f32x4 ww[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            j[q] = ld_quad_nt(col + base + q * kQuadStride);
            ww[q] = ld_quad_nt(w + base + q * kQuadStride);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const f3 xv = ld3(x, j[q][c]);
                ax = fmaf(ww[q][c], xv.x, ax);
                ay = fmaf(ww[q][c], xv.y, ay);
                az = fmaf(ww[q][c], xv.z, az);
            }
        }
    } else {
        for (int q = 0; 4 * q < K; ++q) {
            const i32x4 jq = ld_quad_nt(col + base + q * kQuadStride);
            const f32x4 wq = ld_quad_nt(w + base + q * kQuadStride);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const f3 xv = ld3(x, jq[c]);
                ax = fmaf(wq[c], xv.x, ax);
                ay = fmaf(wq[c], xv.y, ay);
                az = fmaf(wq[c], xv.z, az);
            }
        }
    }
    return f3{ax, ay, az};
}

// ------------------------------------------- compact edge ids (two-pass SpMV)
// The aggregation streams every edge's id and weight once per iteration.  Its
// ids are kept a second time as 16-bit offsets j - i from the row: the k
// nearest lie a few grid cells away, so in the spatially sorted order most
// offsets are small.  Layout: the sliced ELL with octets, row i's slots 8o..8o+7
// in one 16-byte group (int16 element c16_row(i, K) + o * kOctStride + l % 8).
// Slot 0 (always the row itself) holds instead the row's start, within its
// slice, in the list of escaped ids; an offset outside [-32767, 32767] is
// stored as kC16Escape and its id read from that list, which holds a slice's
// escaped ids in row and slot order from c16_base[slice] on.
constexpr int64_t kOctStride = 8 * kSlice;
constexpr int32_t kC16Escape = -32768;
__host__ __device__ inline int c16_k8(int K) { return (K + 7) & ~7; }
__host__ __device__ inline int64_t c16_row(int64_t i, int K) {
    return (i >> 6) * (int64_t)c16_k8(K) * kSlice + (i & (kSlice - 1)) * 8;
}
__host__ __device__ inline int64_t c16_size(int64_t N, int K) { return div_up(N, kSlice) * kSlice * c16_k8(K); }

// Row i's K4 = KT neighbour ids from the compact layout.  Every id, an
// escaped one included, is known before any gather: an escape's position in
// the list follows from the escapes before it in the row.  The row's first
// four escaped ids are read from the four list slots at its start, with no
// branch of their own (the list is as long as the ELL, so p0 + 3 stays
// inside it; slots past the row's own escapes are never selected).
template <int KT>
__device__ __forceinline__ void c16_row_ids(int64_t i, int K, const int16_t* __restrict__ c16,
                                            const uint32_t* __restrict__ c16_base, const int32_t* __restrict__ ovf,
                                            int32_t (&j)[KT]) {
    static_assert(KT % 4 == 0 && KT > 0, "compile-time K4 only");
    constexpr int NO = (KT + 7) / 8;
    const int64_t b16 = c16_row(i, K);
    i32x4 d[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) d[o] = ld_quad_nt(reinterpret_cast<const int32_t*>(c16 + b16 + o * kOctStride));
    const int64_t p0 = (int64_t)c16_base[i >> 6] + (uint32_t)(d[0][0] & 0xffff);
    // more than four escaped ids take a load of their own
    const int32_t e0 = ovf[p0], e1 = ovf[p0 + 1], e2 = ovf[p0 + 2], e3 = ovf[p0 + 3];
    int r = 0;
    j[0] = (int32_t)i;
#pragma unroll
    for (int l = 1; l < KT; ++l) {
        const int32_t word = d[l >> 3][(l & 7) >> 1];
        const int32_t off = (l & 1) ? (word >> 16) : (int32_t)(int16_t)(word & 0xffff);
        int32_t v = (int32_t)(i + off);
        if (off == kC16Escape) {
            v = r == 0 ? e0 : (r == 1 ? e1 : (r == 2 ? e2 : e3));
            if (r >= 4) v = ovf[p0 + r];
            ++r;
        }
        j[l] = v;
    }
}

// The same sum as ell_row_sum<KT> (same slots, same order, same FMAs: bit-
// identical), with the ids decoded from the compact layout.
template <int KT>
__device__ __forceinline__ f3 c16_row_sum(int64_t i, int K, const int16_t* __restrict__ c16,
                                          const uint32_t* __restrict__ c16_base, const int32_t* __restrict__ ovf,
                                          const float* __restrict__ w, const float* __restrict__ x) {
    constexpr int NQ = KT / 4;
    const int64_t base = ell_row(i, K);
    f32x4 ww[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ww[q] = ld_quad_nt(w + base + q * kQuadStride);
    int32_t j[KT];
    c16_row_ids<KT>(i, K, c16, c16_base, ovf, j);
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int l = 0; l < KT; ++l) {
        const f3 xv = ld3(x, j[l]);
        const float wl = ww[l >> 2][l & 3];
        ax = fmaf(wl, xv.x, ax);
        ay = fmaf(wl, xv.y, ay);
        az = fmaf(wl, xv.z, az);
    }
    return f3{ax, ay, az};
}

// Compile-time K4 for the common neighbour counts, else runtime.
template <class F>
__host__ __device__ inline void dispatch_k4(int K, F&& go) {
    switch (ell_k4(K)) {
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 12: go(std::integral_constant<int, 12>{}); break;
    case 16: go(std::integral_constant<int, 16>{}); break;
    case 20: go(std::integral_constant<int, 20>{}); break;
    case 24: go(std::integral_constant<int, 24>{}); break;
    case 28: go(std::integral_constant<int, 28>{}); break;
    case 32: go(std::integral_constant<int, 32>{}); break;
    default: go(std::integral_constant<int, 0>{}); break;
    }
}

// Henyey-Greenstein density as a function of u = 1 - cos between unit
// vectors, u = |a - b|^2 / 2:  HG = (1-g^2) / (4 pi ((1-g)^2 + 2 g u)^(3/2)).
struct HG {
    float c;    // (1 - g^2) / (4 pi)
    float a;    // (1 - g)^2
    float two_g;
    __host__ __device__ static HG make(float g) {
        HG h;
        h.c = (1.0f - g * g) / (4.0f * kPi);
        h.a = (1.0f - g) * (1.0f - g);
        h.two_g = 2.0f * g;
        return h;
    }
    __device__ float operator()(float u) const {
        float den = fmaf(two_g, u, a);
        float r = __frsqrt_rn(den);
        return c * r * r * r;
    }
};

__device__ inline float one_minus_cos(f3 a, f3 b) {
    float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return 0.5f * fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// The pixel's direct term from the extra first-vertex emitter samples of
// path p (paths->n_extra = M > 0): (1/M) sum_m (rho(sun) Ls_m + rho(we_m)
// Le_m / env_pdf), rho about the first vertex's arriving direction t; with
// dg != NULL also its derivative with respect to g (rho h, h = d ln HG/dg).
__device__ inline float hg_dlog(float g, float u);
template <class Rho>
__device__ inline f3 extra_direct(const pg_paths& P, int64_t p, int64_t v0, f3 t, const Rho& rho, float g, f3 sun,
                                  float env_pdf, f3* dg) {
    const int M = P.n_extra;
    const float us = one_minus_cos(t, sun);
    const float rs = rho(us), hs = dg ? hg_dlog(g, us) : 0.0f;
    f3 d{0.f, 0.f, 0.f}, e{0.f, 0.f, 0.f};
    for (int m = 0; m < M; ++m) {
        const int64_t o = ((int64_t)p * M + m) * 3;
        const f3 we{P.fb_dir_env[o], P.fb_dir_env[o + 1], P.fb_dir_env[o + 2]};
        const float u = one_minus_cos(t, we);
        const float re = rho(u) / env_pdf;
        d.x += rs * P.fb_l_sun[o] + re * P.fb_l_env[o];
        d.y += rs * P.fb_l_sun[o + 1] + re * P.fb_l_env[o + 1];
        d.z += rs * P.fb_l_sun[o + 2] + re * P.fb_l_env[o + 2];
        if (dg) {
            const float he = hg_dlog(g, u);
            e.x += rs * hs * P.fb_l_sun[o] + re * he * P.fb_l_env[o];
            e.y += rs * hs * P.fb_l_sun[o + 1] + re * he * P.fb_l_env[o + 1];
            e.z += rs * hs * P.fb_l_sun[o + 2] + re * he * P.fb_l_env[o + 2];
        }
    }
    const float inv = 1.0f / (float)M;
    d = f3{d.x * inv, d.y * inv, d.z * inv};
    e = f3{e.x * inv, e.y * inv, e.z * inv};
    if (P.dir_pl) {   // a point light keeps the vertex's own shadow-ray sample
        const float u = one_minus_cos(t, f3{P.dir_pl[3 * v0], P.dir_pl[3 * v0 + 1], P.dir_pl[3 * v0 + 2]});
        const float rp = rho(u), hp = dg ? rp * hg_dlog(g, u) : 0.0f;
        d.x += rp * P.l_pl[3 * v0];
        d.y += rp * P.l_pl[3 * v0 + 1];
        d.z += rp * P.l_pl[3 * v0 + 2];
        e.x += hp * P.l_pl[3 * v0];
        e.y += hp * P.l_pl[3 * v0 + 1];
        e.z += hp * P.l_pl[3 * v0 + 2];
    }
    if (dg) *dg = e;
    return d;
}

// d ln HG / d g at u:  -2g/(1-g^2) - 3 (g - cos) / ((1-g)^2 + 2 g u).
__device__ inline float hg_dlog(float g, float u) {
    float den = fmaf(2.0f * g, u, (1.0f - g) * (1.0f - g));
    return -2.0f * g / (1.0f - g * g) - 3.0f * (g - (1.0f - u)) / den;
}

// Cell-centred trilinear interpolation weights on an R^3 grid ([z][y][x]):
// per axis u = R x - 0.5, i0 = floor(u), f = u - i0; corner indices i0 and
// i0+1 are each clamped to [0, R-1], the weights (1-f, f) are kept.
__device__ inline void trilerp_corners(int R, float px, float py, float pz, uint32_t idx[8], float w[8]) {
    const float p[3] = {px, py, pz};
    int lo[3], hi[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float u = (float)R * p[a] - 0.5f;
        float fl = floorf(u);
        f[a] = u - fl;
        int l = (int)fl;
        lo[a] = min(max(l, 0), R - 1);
        hi[a] = min(max(l + 1, 0), R - 1);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        const uint32_t ix = bx ? hi[0] : lo[0], iy = by ? hi[1] : lo[1], iz = bz ? hi[2] : lo[2];
        idx[c] = (iz * (uint32_t)R + iy) * (uint32_t)R + ix;
        w[c] = (bx ? f[0] : 1.0f - f[0]) * (by ? f[1] : 1.0f - f[1]) * (bz ? f[2] : 1.0f - f[2]);
    }
}

// Appends one item for every active lane with `take` set to a list whose
// length is *counter and returns the lane's slot (meaningful where take is
// set): one atomic per wave for the wave's total, each lane's offset from a
// ballot and the count of taking lanes below it.  All active lanes of the wave
// must call it together.
__device__ inline uint32_t wave_append(uint32_t* counter, bool take) {
    const uint64_t m = __ballot(take);
    if (m == 0) return 0;
    const int lane = (int)__lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader, kWave);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Record a device-detected input error (flag may be NULL).
__device__ inline void set_flag(int32_t* flag, int32_t bit) {
    if (flag) atomicOr(flag, bit);
}

// Calls go(std::integral_constant<int, KP>) with KP the smallest power of two >= K.
template <typename F>
inline void dispatch_kp(int K, F&& go) {
    if (K <= 1) go(std::integral_constant<int, 1>{});
    else if (K <= 2) go(std::integral_constant<int, 2>{});
    else if (K <= 4) go(std::integral_constant<int, 4>{});
    else if (K <= 8) go(std::integral_constant<int, 8>{});
    else if (K <= 16) go(std::integral_constant<int, 16>{});
    else if (K <= 32) go(std::integral_constant<int, 32>{});
    else go(std::integral_constant<int, 64>{});
}

// Sum over aligned groups of KP lanes (KP a power of two <= 64).
template <int KP>
__device__ inline float group_sum(float v) {
#pragma unroll
    for (int o = KP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Vertex record in the internal (spatially sorted) order: everything the
// aggregation step reads about a neighbour, 80 bytes, 16-byte aligned.
struct alignas(16) VRec {
    float t[3];      // dir_in
    float w[3];      // dir_out
    float we[3];     // dir_env
    float ls[3];     // l_sun
    float le[3];     // l_env
    float lp[3];     // l_phase
    float alpha;     // albedo
    float pad;
};
static_assert(sizeof(VRec) == 80, "VRec layout");

// Uniform method constants for the kernels.
struct Consts {
    HG rho;          // receiver phase (g)
    HG pdf;          // sampling pdf (g_s)
    float g;
    float env_pdf;
    f3 sun;
    int32_t K;
    int32_t init;
    int32_t final_gather;
};

// ------------------------------------------------------- launch wrappers ---
// Each returns hipSuccess or the launch error.  All take the stream last.

// grid build: quantise + histogram, exclusive scan, scatter into cell order
hipError_t launch_quantize_count(int64_t N, const float* pos, int shift, uint32_t* count, uint32_t* cellid,
                                 uint32_t* rank, int32_t* flag, hipStream_t s);
size_t scan_partials_bytes(int64_t n);
hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                                 hipStream_t s);
hipError_t launch_scatter(int64_t N, const pg_paths& paths, int shift, const uint32_t* cellid,
                          const uint32_t* rank, const uint32_t* cell_start, int32_t* perm, int32_t* inv,
                          uint64_t* qsorted, VRec* rec, hipStream_t s);
// redo: [N] scratch list, nredo: one counter (queries the fast 64-bit-key
// search hands to the exact one)
hipError_t launch_cell_range(int64_t ncells, int shift, const uint32_t* start, uint2* range, hipStream_t s);
hipError_t launch_knn(int64_t N, int K, int shift, const uint64_t* qsorted, const int32_t* perm,
                      const int32_t* inv, const uint2* cell_range, int32_t* col_sorted, int32_t* col_canon,
                      int64_t* row_ptr, uint32_t* redo, uint32_t* nredo, bool exact_only, hipStream_t s);

// records in path order (no permutation)
hipError_t launch_pack_records(int64_t N, const pg_paths& paths, VRec* rec, int32_t* flag, hipStream_t s);

// aggregation operators (edge weights, direct terms) in the records' id
// space, into the sliced-ELL layout (ell = 1, the internal render) or a
// row-major CSR (ell = 0, the pg_edges entry point).  canon_row (nullable)
// maps local row -> path-order row for the optional path-order outputs.
struct EdgeOut {
    int ell;             // 1: col / w / gw in the sliced-ELL layout, 0: row-major
    float* w;            // local order (required): ell_size(N, K) or N*K elements
    float* gw;           // dw/dg in the same layout, or NULL
    float* b;            // [N] f3 local
    float* dpt;          // [N] f3 local
    float* r;            // [N] local
    float* alpha;        // [N] local
    const int32_t* canon_row;
    const float* emit;   // volume emission e, [N] f3 in canonical (path) order, nullable
    const float* dir_pl; // point light (canonical order), nullable
    const float* l_pl;
    float* w_ind;        // path order, nullable
    float* w_ph;
    float* w_env;
    float* b_canon;
    float* dpt_canon;
};
hipError_t launch_edges(int64_t N, const Consts& c, const int32_t* col, const VRec* rec, const EdgeOut& o,
                        int32_t* flag, hipStream_t s);

// per-path pass: successor / predecessor in local ids and the initial L
hipError_t launch_paths(int64_t P, int64_t N, const int64_t* off, const int32_t* inv, const float* alpha,
                        const float* dpt, const float* r, const float* emit, int init, int32_t* succ, int32_t* pred,
                        float* x0,
                        int32_t* flag, hipStream_t s);

// propagation
hipError_t launch_spmv(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                       const float* alpha, float* y, hipStream_t s);
// the same product over the sliced-ELL layout, one thread per row
// (tile: workgroup size, tile_group: consecutive tiles per XCD; 0 = defaults)
hipError_t launch_spmv_ell(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                           const float* alpha, const int32_t* rowmask, float* y, hipStream_t s, int tile = 0,
                           int tile_group = 0);
// aggregation fused with propagation: row i's result goes to x_new[pred i];
// rows without a predecessor are skipped
hipError_t launch_spmv_scatter(int64_t N, int K, const int32_t* col, const float* w, const float* x,
                               const float* b, const float* alpha, const int32_t* pred, float* xn, hipStream_t s);
hipError_t launch_shift(int64_t N, const int32_t* succ, const float* y, float* x, hipStream_t s, int tile = 0);
hipError_t launch_check_rows(int64_t N, int K, const int64_t* row_ptr, int32_t* flag, hipStream_t s);
// compact ids of the sliced ELL (see c16_row_sum): c16 [c16_size], c16_base
// [n_slices + 1], ovf [ell_size] (room for every id), cnt / partials scratch
hipError_t launch_c16_build(int64_t N, int K, const int32_t* col, int16_t* c16, uint32_t* cnt, uint32_t* c16_base,
                            uint32_t* partials, int32_t* ovf, hipStream_t s);
hipError_t launch_spmv_c16(int64_t N, int K, const int16_t* c16, const uint32_t* c16_base, const int32_t* ovf,
                           const int32_t* col, const float* w, const float* x, const float* b, const float* alpha,
                           float* y, hipStream_t s, int tile = 0, int tile_group = 0);
hipError_t launch_shifted_build(int64_t N, int K, const int32_t* succ, const int32_t* col, const float* w,
                                const float* b, const float* alpha, int32_t* mcol, float* mw, float* c,
                                hipStream_t s);
hipError_t launch_spmv_shifted(int64_t N, int K, const int32_t* succ, const int32_t* mcol, const float* mw,
                               const float* c, const float* x, float* xn, hipStream_t s);

// output to pixels; inv (nullable) maps path-order vertex -> local id; with
// inv the edges are in the sliced-ELL layout, without it row-major
hipError_t launch_pixels(const pg_paths& paths, const Consts& c, const int32_t* inv, const int32_t* col,
                         const float* w, const float* x, const float* dpt, const float* r, const float* alpha,
                         float* image, int32_t* flag, hipStream_t s);

// small utilities
hipError_t launch_permute3(int64_t N, const int32_t* idx, const float* src, float* dst, int gather,
                           hipStream_t s);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);
hipError_t launch_fill_value(void* p, size_t bytes, uint32_t v, hipStream_t s);
hipError_t launch_alpha(int64_t N, const pg_paths& paths, float* alpha, hipStream_t s);

}  // namespace pg
