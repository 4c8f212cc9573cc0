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
template <int KT, bool SCATTER, int BS>
__global__ __launch_bounds__(BS) void k_spmv_ell(int64_t N, int K, const int32_t* __restrict__ col,
                                                 const float* __restrict__ w, const float* __restrict__ x,
                                                 const float* __restrict__ b, const float* __restrict__ alpha,
                                                 const int32_t* __restrict__ rowmask, float* __restrict__ y,
                                                 int group) {
    const int64_t tile = grouped_tile(blockIdx.x, gridDim.x, group);
    const int64_t i = tile * BS + threadIdx.x;
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
                        const float* alpha, const int32_t* rowmask, float* y, hipStream_t s, int tile, int group) {
    dispatch_tile(tile, [&](auto bs) {
        constexpr int BS = decltype(bs)::value;
        dim3 grid((unsigned)div_up(N, BS)), block(BS);
        dispatch_k4(K, [&](auto kt) {
            constexpr int KT = decltype(kt)::value;
            hipLaunchKernelGGL((k_spmv_ell<KT, SCATTER, BS>), grid, block, 0, s, N, K, col, w, x, b, alpha, rowmask,
                               y, group);
        });
    });
}

hipError_t launch_spmv_ell(int64_t N, int K, const int32_t* col, const float* w, const float* x, const float* b,
                           const float* alpha, const int32_t* rowmask, float* y, hipStream_t s, int tile,
                           int tile_group) {
    if (N == 0) return hipSuccess;
    go_spmv_ell<false>(N, K, col, w, x, b, alpha, rowmask, y, s, tile, tile_group);
    return hipGetLastError();
}

hipError_t launch_spmv_scatter(int64_t N, int K, const int32_t* col, const float* w, const float* x,
                               const float* b, const float* alpha, const int32_t* pred, float* xn, hipStream_t s) {
    if (N == 0) return hipSuccess;
    go_spmv_ell<true>(N, K, col, w, x, b, alpha, pred, xn, s, 0, 0);
    return hipGetLastError();
}

// ------------------------------------------------- compact edge ids ---
// One wave per 64-row slice: each lane counts its row's escaped offsets, a
// wave prefix sum gives the row's start in the slice's escape list (slot 0),
// and the row's octets are written as 16-byte stores.  Rows past N keep
// offset 0 in every slot.
__global__ __launch_bounds__(kBlock) void k_c16_build(int64_t N, int K, const int32_t* __restrict__ col,
                                                      int16_t* __restrict__ c16, uint32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nsl = div_up(N, kSlice);
    if ((i >> 6) >= nsl) return;   // whole waves leave together (a slice is one wave)
    const int K4 = ell_k4(K), K8 = c16_k8(K);
    uint32_t n = 0;
    if (i < N)
        for (int l = 1; l < K4; ++l) {
            const int64_t off = (int64_t)col[eidx(i, l, K)] - i;
            n += (off < -32767 || off > 32767) ? 1u : 0u;
        }
    uint32_t inc = n;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    const uint32_t start = inc - n;
    const int64_t b16 = c16_row(i, K);
    for (int o = 0; 8 * o < K8; ++o) {
        int32_t words[4];
        for (int h = 0; h < 4; ++h) {
            int32_t v[2];
            for (int e = 0; e < 2; ++e) {
                const int l = 8 * o + 2 * h + e;
                int32_t val = 0;
                if (l == 0) {
                    val = (int32_t)(start & 0xffffu);
                } else if (i < N && l < K4) {
                    const int64_t off = (int64_t)col[eidx(i, l, K)] - i;
                    val = (off < -32767 || off > 32767) ? kC16Escape : (int32_t)off;
                }
                v[e] = val & 0xffff;
            }
            words[h] = v[0] | (v[1] << 16);
        }
        *reinterpret_cast<i32x4*>(c16 + b16 + o * kOctStride) = i32x4{words[0], words[1], words[2], words[3]};
    }
    if (lane == kWave - 1) cnt[i >> 6] = inc;
}

// Escaped ids of each row at its slice's list start + its slot-0 start.
__global__ __launch_bounds__(kBlock) void k_c16_escapes(int64_t N, int K, const int32_t* __restrict__ col,
                                                        const int16_t* __restrict__ c16,
                                                        const uint32_t* __restrict__ c16_base,
                                                        int32_t* __restrict__ ovf) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    int64_t p = (int64_t)c16_base[i >> 6] + (uint16_t)c16[c16_row(i, K)];
    const int K4 = ell_k4(K);
    for (int l = 1; l < K4; ++l) {
        const int32_t j = col[eidx(i, l, K)];
        const int64_t off = (int64_t)j - i;
        if (off < -32767 || off > 32767) ovf[p++] = j;
    }
}

hipError_t launch_c16_build(int64_t N, int K, const int32_t* col, int16_t* c16, uint32_t* cnt, uint32_t* c16_base,
                            uint32_t* partials, int32_t* ovf, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int64_t nsl = div_up(N, kSlice);
    hipLaunchKernelGGL(k_c16_build, dim3((unsigned)div_up(nsl * kSlice, kBlock)), dim3(kBlock), 0, s, N, K, col,
                       c16, cnt);
    hipError_t e = launch_scan_exclusive(cnt, c16_base, nsl, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_c16_escapes, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, K, col, c16,
                       c16_base, ovf);
    return hipGetLastError();
}

// The two-pass aggregation over the compact ids: the same rows, slots and
// arithmetic as k_spmv_ell, so the same results bit for bit, with 2 bytes per
// id streamed instead of 4 (plus the few escaped ids).
template <int KT, int BS>
__global__ __launch_bounds__(BS) void k_spmv_c16(int64_t N, int K, const int16_t* __restrict__ c16,
                                                 const uint32_t* __restrict__ c16_base,
                                                 const int32_t* __restrict__ ovf, const float* __restrict__ w,
                                                 const float* __restrict__ x, const float* __restrict__ b,
                                                 const float* __restrict__ alpha, float* __restrict__ y, int group) {
    const int64_t tile = grouped_tile(blockIdx.x, gridDim.x, group);
    const int64_t i = tile * BS + threadIdx.x;
    if (i >= N) return;
    const f3 z = c16_row_sum<KT>(i, K, c16, c16_base, ovf, w, x);
    const f3 bb = ld3(b, i);
    const float a = alpha ? alpha[i] : 1.0f;
    st3_nt(y, i, f3{fmaf(a, z.x, bb.x), fmaf(a, z.y, bb.y), fmaf(a, z.z, bb.z)});
}

hipError_t launch_spmv_c16(int64_t N, int K, const int16_t* c16, const uint32_t* c16_base, const int32_t* ovf,
                           const int32_t* col, const float* w, const float* x, const float* b, const float* alpha,
                           float* y, hipStream_t s, int tile, int tile_group) {
    if (N == 0) return hipSuccess;
    if (ell_k4(K) > 32) return launch_spmv_ell(N, K, col, w, x, b, alpha, nullptr, y, s, tile, tile_group);
    dispatch_tile(tile, [&](auto bs) {
        constexpr int BS = decltype(bs)::value;
        dim3 grid((unsigned)div_up(N, BS)), block(BS);
        dispatch_k4(K, [&](auto kt) {
            constexpr int KT = decltype(kt)::value;
            if constexpr (KT > 0)
                hipLaunchKernelGGL((k_spmv_c16<KT, BS>), grid, block, 0, s, N, K, c16, c16_base, ovf, w, x, b, alpha,
                                   y, tile_group);
        });
    });
    return hipGetLastError();
}

// A caller's CSR must have the k-nearest layout, row i = [i K, (i+1) K):
// the kernels of pg_edges / pg_propagate index col and w as i K + l.
__global__ __launch_bounds__(kBlock) void k_check_rows(int64_t N, int K, const int64_t* __restrict__ row_ptr,
                                                       int32_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i <= N && row_ptr[i] != i * (int64_t)K) set_flag(flag, kFlagRows);
}

hipError_t launch_check_rows(int64_t N, int K, const int64_t* row_ptr, int32_t* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_rows, dim3((unsigned)div_up(N + 1, kBlock)), dim3(kBlock), 0, s, N, K, row_ptr,
                       flag);
    return hipGetLastError();
}

// L(v) = y(succ v), 0 at a path's end.  Two vertices per thread, strided by
// the grid so every access stays coalesced, for two independent gathers; the
// successor ids (read once) are streamed and L is stored non-temporally.
// Every load is unconditional (indices clamped to a valid element, the value
// masked afterwards), so both successor ids and then both gathers are in
// flight together instead of each waiting at a branch.
constexpr int kShiftPer = 2;
template <int BS>
__global__ __launch_bounds__(BS) void k_shift(int64_t N, const int32_t* __restrict__ succ,
                                              const float* __restrict__ y, float* __restrict__ x) {
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t v0 = tile * (int64_t)BS * kShiftPer + threadIdx.x;
    int32_t u[kShiftPer];
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) {
        const int64_t v = v0 + (int64_t)k * BS;
        u[k] = __builtin_nontemporal_load(succ + (v < N ? v : N - 1));
    }
    f3 val[kShiftPer];
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) val[k] = ld3(y, u[k] > 0 ? u[k] : 0);
    // an empty asm that takes every gathered value keeps the compiler from
    // sinking one vertex's loads into its guarded store (which serialises
    // the two load chains)
    asm volatile("" ::"v"(val[0].x), "v"(val[0].y), "v"(val[0].z), "v"(val[1].x), "v"(val[1].y), "v"(val[1].z));
    static_assert(kShiftPer == 2, "the asm above names two vertices");
#pragma unroll
    for (int k = 0; k < kShiftPer; ++k) {
        const int64_t v = v0 + (int64_t)k * BS;
        if (u[k] < 0) val[k] = f3{0.f, 0.f, 0.f};
        if (v < N) st3_nt(x, v, val[k]);
    }
}

hipError_t launch_shift(int64_t N, const int32_t* succ, const float* y, float* x, hipStream_t s, int tile) {
    if (N == 0) return hipSuccess;
    dispatch_tile(tile, [&](auto bs) {
        constexpr int BS = decltype(bs)::value;
        hipLaunchKernelGGL(k_shift<BS>, dim3((unsigned)div_up(N, (int64_t)BS * kShiftPer)), dim3(BS), 0, s, N,
                           succ, y, x);
    });
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
