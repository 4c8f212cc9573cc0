// pg_prop.hip -- iterated aggregation + propagation and the output to pixels.
//
// Paper eqs. ag-mf, rte-pg and rte-mff: the indirect part of the scattered
// radiance is re-aggregated from the neighbours' incoming indirect radiance,
// the constant direct part is added, and the result is propagated one edge
// back along each path.  With delta tracking the propagation factor
// transmittance / free-flight pdf equals 1/sigma_t at the collision, which
// turns sigma_s * phase into albedo * phase, so propagation is a shift:
//   y_i = b_i + albedo_i sum_j w_ij L(j),   L(v) = y(succ v), 0 at a path's end.
//
// Two schedules, identical arithmetic:
//  * two-pass: a sparse matrix-vector product over the spatially sorted rows
//    (neighbour gathers stay within a few grid cells), then the shift as one
//    gather per vertex;
//  * shifted: the rows are pre-arranged in predecessor order, row v holding
//    albedo_u w_u. and b_u of its successor u, so one pass per iteration
//    computes L directly.
// Both are sparse gathers bound by HBM bandwidth (about 0.5 flop per byte).
#include "pg_internal.h"

namespace pg {

// One group of KP lanes per row, lane = edge: the row's column ids and
// weights are read as contiguous, coalesced segments, each lane gathers one
// x value, and the group reduces.  alpha == NULL means 1.
template <int KP>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t N, int K, const int32_t* __restrict__ col,
                                                 const float* __restrict__ w, const float* __restrict__ x,
                                                 const float* __restrict__ b, const float* __restrict__ alpha,
                                                 const int32_t* __restrict__ rowmask, float* __restrict__ y) {
    constexpr int GR = kBlock / KP;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % KP;
    const int64_t i = tile * GR + threadIdx.x / KP;
    const bool row_ok = i < N && (!rowmask || rowmask[i] >= 0);
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    if (row_ok && lane < K) {
        const int64_t e = i * K + lane;
        const int64_t j = col[e];
        const float ww = w[e];
        if ((uint64_t)j < (uint64_t)N) {   // ids from callers are not trusted
            ax = ww * x[3 * j];
            ay = ww * x[3 * j + 1];
            az = ww * x[3 * j + 2];
        }
    }
    ax = group_sum<KP>(ax);
    ay = group_sum<KP>(ay);
    az = group_sum<KP>(az);
    if (i < N && lane == 0) {
        if (row_ok) {
            const float a = alpha ? alpha[i] : 1.0f;
            y[3 * i] = fmaf(a, ax, b[3 * i]);
            y[3 * i + 1] = fmaf(a, ay, b[3 * i + 1]);
            y[3 * i + 2] = fmaf(a, az, b[3 * i + 2]);
        } else {
            y[3 * i] = 0.0f;
            y[3 * i + 1] = 0.0f;
            y[3 * i + 2] = 0.0f;
        }
    }
}

hipError_t launch_spmv(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                       const float* alpha, float* y, hipStream_t s) {
    if (N == 0) return hipSuccess;
    dispatch_kp(K, [&](auto kp) {
        constexpr int KP = decltype(kp)::value;
        hipLaunchKernelGGL(k_spmv<KP>, dim3((unsigned)div_up(N, kBlock / KP)), dim3(kBlock), 0, s, N, K, col, w,
                           x, b, alpha, (const int32_t*)nullptr, y);
    });
    return hipGetLastError();
}

// One thread per row over the sliced-ELL layout: each wave owns one slice of
// 64 rows and reads four edges of each of its rows per 16-byte load (1 KiB
// contiguous per wave).  rowmask (nullable): rows with rowmask[i] < 0 output
// 0.  alpha NULL means 1.  SCATTER: the row's result is stored at
// y[rowmask[i]] (the predecessor) and rows with rowmask[i] < 0 are skipped;
// otherwise such rows store 0 at y[i].
//
// Blocks run in plain launch order (all XCDs sweep the same region of the
// sorted rows together, which measured faster here than giving each XCD its
// own contiguous range), and the edge ids and weights, read exactly once, are
// loaded non-temporally so they do not displace the gathered vector in L2.
template <int KT, bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_spmv_ell(int64_t N, int K, const int32_t* __restrict__ col,
                                                     const float* __restrict__ w, const float* __restrict__ x,
                                                     const float* __restrict__ b, const float* __restrict__ alpha,
                                                     const int32_t* __restrict__ rowmask, float* __restrict__ y) {
    const int64_t tile = blockIdx.x;
    const int64_t i = tile * kBlock + threadIdx.x;
    if (i >= N) return;
    int64_t dst = i;
    if (rowmask) {
        dst = rowmask[i];
        if (dst < 0) {
            if (!SCATTER) st3(y, i, f3{0.f, 0.f, 0.f});
            return;
        }
        if (!SCATTER) dst = i;
    }
    const f3 z = ell_row_sum<KT>(i, K, col, w, x);
    const f3 bb = ld3(b, i);
    const float a = alpha ? alpha[i] : 1.0f;
    st3_nt(y, dst, f3{fmaf(a, z.x, bb.x), fmaf(a, z.y, bb.y), fmaf(a, z.z, bb.z)});
}

template <bool SCATTER>
static void go_spmv_ell(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                        const float* alpha, const int32_t* rowmask, float* y, hipStream_t s) {
    dim3 grid((unsigned)div_up(N, kBlock)), block(kBlock);
    dispatch_k4(K, [&](auto kt) {
        constexpr int KT = decltype(kt)::value;
        hipLaunchKernelGGL((k_spmv_ell<KT, SCATTER>), grid, block, 0, s, N, K, col, w, x, b, alpha, rowmask, y);
    });
}

hipError_t launch_spmv_ell(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                           const float* alpha, const int32_t* rowmask, float* y, hipStream_t s) {
    if (N == 0) return hipSuccess;
    go_spmv_ell<false>(N, K, col, w, x, b, alpha, rowmask, y, s);
    return hipGetLastError();
}

hipError_t launch_spmv_scatter(int64_t N, int K, const int32_t* col, const float* w, const float* x,
                               const float* b, const float* alpha, const int32_t* pred, float* xn, hipStream_t s) {
    if (N == 0) return hipSuccess;
    go_spmv_ell<true>(N, K, col, w, x, b, alpha, pred, xn, s);
    return hipGetLastError();
}

// L(v) = y(succ v), 0 at a path's end.  Two vertices per thread, strided by
// the grid so every access stays coalesced, for two independent gathers; the
// successor ids (read once) are streamed and L is stored non-temporally.
constexpr int kShiftPer = 2;
__global__ __launch_bounds__(kBlock) void k_shift(int64_t N, const int32_t* __restrict__ succ,
                                                  const float* __restrict__ y, float* __restrict__ x) {
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t v0 = tile * (int64_t)kBlock * kShiftPer + threadIdx.x;
    int64_t u[kShiftPer];
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) {
        const int64_t v = v0 + (int64_t)k * kBlock;
        u[k] = v < N ? (int64_t)__builtin_nontemporal_load(succ + v) : -1;
    }
    f3 val[kShiftPer];
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) val[k] = u[k] >= 0 ? ld3(y, u[k]) : f3{0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) {
        const int64_t v = v0 + (int64_t)k * kBlock;
        if (v < N) st3_nt(x, v, val[k]);
    }
}

hipError_t launch_shift(int64_t N, const int32_t* succ, const float* y, float* x, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shift, dim3((unsigned)div_up(N, (int64_t)kBlock * kShiftPer)), dim3(kBlock), 0, s, N,
                       succ, y, x);
    return hipGetLastError();
}

// Row v of the shifted operator = albedo_u * row u of W, constant c_v = b_u,
// u = succ(v); a row without successor keeps zero weights (self columns).
// All slots of the row's quads are written (the padding slots of W hold
// (u, 0), so they become weight-0 slots here too).
__global__ __launch_bounds__(kBlock) void k_shifted_build(int64_t N, int K, const int32_t* __restrict__ succ,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ w, const float* __restrict__ b,
                                                          const float* __restrict__ alpha,
                                                          int32_t* __restrict__ mcol, float* __restrict__ mw,
                                                          float* __restrict__ c) {
    const int K4 = ell_k4(K);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * (int64_t)K4) return;
    const int64_t v = t / K4;
    const int k = (int)(t - v * K4);
    const int64_t u = succ[v];
    const int64_t e = eidx(v, k, K);
    if (u >= 0) {
        mcol[e] = col[eidx(u, k, K)];
        mw[e] = alpha[u] * w[eidx(u, k, K)];
    } else {
        mcol[e] = (int32_t)v;
        mw[e] = 0.0f;
    }
    if (k == 0) st3(c, v, u >= 0 ? ld3(b, u) : f3{0.f, 0.f, 0.f});
}

hipError_t launch_shifted_build(int64_t N, int K, const int32_t* succ, const int32_t* col, const float* w,
                                const float* b, const float* alpha, int32_t* mcol, float* mw, float* c,
                                hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shifted_build, dim3((unsigned)div_up(N * (int64_t)ell_k4(K), kBlock)), dim3(kBlock), 0, s,
                       N, K, succ, col, w, b, alpha, mcol, mw, c);
    return hipGetLastError();
}

hipError_t launch_spmv_shifted(int64_t N, int K, const int32_t* succ, const int32_t* mcol, const float* mw,
                               const float* c, const float* x, float* xn, hipStream_t s) {
    return launch_spmv_ell(N, K, mcol, mw, x, c, nullptr, succ, xn, s);
}

// ------------------------------------------------------------- pixels ---
// One thread per pixel; its spp paths are consecutive.  o_p as in the
// "Final output" paragraph with the non-aggregated direct term at the first
// vertex ("Handling direct Light") -- or the estimate of the extra samples
// recorded there -- and that vertex's volume emission.  inv == NULL: local ids are path-order
// ids; r == NULL / alpha == NULL: computed from the path records.
__global__ __launch_bounds__(kBlock) void k_pixels(pg_paths P, Consts c, const int32_t* __restrict__ inv,
                                                   const int32_t* __restrict__ col, const float* __restrict__ w,
                                                   const float* __restrict__ x, const float* __restrict__ dpt,
                                                   const float* __restrict__ r, const float* __restrict__ alpha,
                                                   float* __restrict__ image, int32_t* flag) {
    const int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)P.width * P.height;
    if (px >= npix) return;
    const int64_t N = P.n_vertices;
    const int K = c.K;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int k = 0; k < P.spp; ++k) {
        const int64_t p = px * P.spp + k;
        sx += P.e_cam[3 * p];
        sy += P.e_cam[3 * p + 1];
        sz += P.e_cam[3 * p + 2];
        const int64_t a = P.path_offsets[p], e = P.path_offsets[p + 1];
        if (e <= a) continue;
        if (a < 0 || e > N) {
            set_flag(flag, kFlagOffsets);
            continue;
        }
        const int64_t s0 = inv ? (int64_t)inv[a] : a;
        float ix = 0.0f, iy = 0.0f, iz = 0.0f;
        if (c.final_gather == 0) {
            for (int l = 0; l < K; ++l) {
                const int64_t e = inv ? eidx(s0, l, K) : s0 * K + l;
                const int64_t j = col[e];
                if (j < 0 || j >= N) {
                    set_flag(flag, kFlagIndex);
                    continue;
                }
                const float ww = w[e];
                ix = fmaf(ww, x[3 * j], ix);
                iy = fmaf(ww, x[3 * j + 1], iy);
                iz = fmaf(ww, x[3 * j + 2], iz);
            }
        } else {
            float rr;
            if (r) {
                rr = r[s0];
            } else {
                const f3 t = ld3(P.dir_in, a), wo = ld3(P.dir_out, a);
                const float u = one_minus_cos(t, wo);
                rr = c.rho(u) / c.pdf(u);
            }
            ix = rr * x[3 * s0];
            iy = rr * x[3 * s0 + 1];
            iz = rr * x[3 * s0 + 2];
        }
        float al;
        if (alpha) {
            al = alpha[s0];
        } else if (P.albedo_grid) {
            uint32_t idx[8];
            float tw[8];
            trilerp_corners(P.albedo_grid_res, P.pos[3 * a], P.pos[3 * a + 1], P.pos[3 * a + 2], idx, tw);
            al = 0.0f;
            for (int q = 0; q < 8; ++q) al = fmaf(tw[q], P.albedo_grid[idx[q]], al);
        } else {
            al = P.albedo[a];
        }
        if (P.l_emit) {   // volume emission of the first vertex, seen by the camera unscattered
            sx += P.l_emit[3 * a];
            sy += P.l_emit[3 * a + 1];
            sz += P.l_emit[3 * a + 2];
        }
        f3 dd = ld3(dpt, s0);
        if (P.n_extra > 0) dd = extra_direct(P, p, a, ld3(P.dir_in, a), c.rho, c.g, c.sun, c.env_pdf, nullptr);
        sx = fmaf(al, dd.x + ix, sx);
        sy = fmaf(al, dd.y + iy, sy);
        sz = fmaf(al, dd.z + iz, sz);
    }
    const float inv_spp = 1.0f / (float)P.spp;
    image[3 * px] = sx * inv_spp;
    image[3 * px + 1] = sy * inv_spp;
    image[3 * px + 2] = sz * inv_spp;
}

hipError_t launch_pixels(const pg_paths& paths, const Consts& c, const int32_t* inv, const int32_t* col,
                         const float* w, const float* x, const float* dpt, const float* r, const float* alpha,
                         float* image, int32_t* flag, hipStream_t s) {
    const int64_t npix = (int64_t)paths.width * paths.height;
    if (npix == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pixels, dim3((unsigned)div_up(npix, kBlock)), dim3(kBlock), 0, s, paths, c, inv, col, w,
                       x, dpt, r, alpha, image, flag);
    return hipGetLastError();
}

// ----------------------------------------------------------- utilities ---

// gather:  dst[i] = src[idx[i]];  scatter: dst[idx[i]] = src[i]   (float3 rows)
__global__ __launch_bounds__(kBlock) void k_permute3(int64_t N, const int32_t* __restrict__ idx,
                                                     const float* __restrict__ src, float* __restrict__ dst,
                                                     int gather) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t j = idx[i];
    if (gather) st3(dst, i, ld3(src, j));
    else st3(dst, j, ld3(src, i));
}

hipError_t launch_permute3(int64_t N, const int32_t* idx, const float* src, float* dst, int gather,
                           hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute3, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, idx, src, dst,
                       gather);
    return hipGetLastError();
}

// Fill bytes with a 32-bit pattern (a kernel, not a memset node, so the
// sequence can be captured in a graph).
__global__ __launch_bounds__(kBlock) void k_fill(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)div_up(n, kBlock)), dim3(kBlock), 0, s, (uint32_t*)p, n, 0u);
    return hipGetLastError();
}

hipError_t launch_fill_value(void* p, size_t bytes, uint32_t v, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)div_up(n, kBlock)), dim3(kBlock), 0, s, (uint32_t*)p, n, v);
    return hipGetLastError();
}

}  // namespace pg
