// pg_backward.hip -- reverse mode of the render with respect to the albedo
// (per vertex and through a trilinear grid) and the receiver-side HG
// parameter g, with the recorded paths and the sampling pdfs held fixed.
//
// Every kernel reverses one forward step, in the opposite order:
//   output to pixels  ->  D reverse sweeps (shift^T, then aggregation^T with
//   the transposed CSR)  ->  path-traced initial estimate (forward walk)  ->
//   direct terms and the g-dependence of every phase evaluation  ->
//   trilinear scatter of d/d albedo into the grid.
// d rho / d g = rho * h(u),  h = d ln HG / d g.  Block partial sums of dL/dg
// go to fixed slots and are reduced in a fixed order, so for one sorted layout
// dL/dg does not depend on scheduling; the grid scatter and the output's
// neighbour scatter use float atomics (order-dependent in the last bits).
// The sorted layout itself follows the grid's atomic in-cell order, so the
// reverse sums' order, and the gradients' last bits, can change between runs.
#include <utility>

#include "pg_api_common.h"

namespace pg {


// ------------------------------------------------- transposed operator ---
// W^T in a sliced ELL over permuted T-rows (the SELL-C-sigma layout of
// Kreutzer et al., 2014, with C = 64 and sigma = kTWin): within each window
// of kTWin consecutive vertices, the T-rows (T-row j: the rows i that have j
// as a neighbour) are ordered by decreasing in-degree, ties by vertex, and
// T-row j takes position tpos[j] (trow is the inverse).  Position r lives in
// slice r/64; an entry is (source row, weight) in 8 bytes (one load each in
// the transposed product; the build's passes move one word instead of two:
// build 14.1 -> 12.0 ms at 22M vertices, the product within 1%); entry q of
// a slice's 64 T-rows is contiguous, and a slice is as
// long as its longest T-row, capped at `cap` entries.  On k-nearest-neighbour
// graphs the padding is about 45% of the entries with slices of consecutive
// vertices and about 26% with windows of 128.  Wider windows pad less (4% at
// 1024) but spread a wave's lanes over more vertices, whose z-bar gathers
// then share fewer cache lines: the transposed product was 5% faster at 128,
// 2% at 256, and 18% and 42% slower at 512 and 1024.  Entries past the
// cap go to an overflow list of (j, i, w) applied with atomics (none for
// ordinary neighbour graphs; degenerate inputs such as many coincident points
// can have a few).
//
// The reverse sweep keeps the adjoint lam of L_t in position order, so the
// transposed product writes it contiguously: the row kernel reads it through
// ppred (the predecessor's position), the output and path-traced adjoints
// through tpos.
//
// Built in six passes: in-degrees with atomics, which also give every edge
// its arrival rank at its T-row (one byte); the windows' order; slice lengths
// and their scan; every edge stored at its rank (no atomics); each T-row
// sorted by source row in registers, so the reverse sums run in a fixed order
// for a given sorted layout; the predecessors' positions.

// Row i and slot l of ELL position e (inverse of eidx); l >= K is padding.
__device__ inline void ell_slot(int64_t e, int K, int64_t& i, int& l) {
    const int64_t per_slice = (int64_t)ell_k4(K) * kSlice;
    const int64_t sl = e / per_slice, off = e - sl * per_slice;
    const int q = (int)(off / kQuadStride), in = (int)(off - (int64_t)q * kQuadStride);
    i = sl * kSlice + (in >> 2);
    l = 4 * q + (in & 3);
}

// in-degree, and each edge's arrival rank at its T-row (255 = past any cap);
// one thread per ELL position, in storage order.
__global__ __launch_bounds__(kBlock) void k_tcount(int64_t N, int K, int64_t EL, const int32_t* __restrict__ col,
                                                   uint32_t* __restrict__ cnt, uint8_t* __restrict__ rank) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= EL) return;
    int64_t i;
    int l;
    ell_slot(e, K, i, l);
    if (i >= N || l >= K) return;
    const uint32_t q = atomicAdd(&cnt[col[e]], 1u);
    rank[e] = (uint8_t)(q < 255u ? q : 255u);
}

// The same counts and ranks with most atomics in LDS.  A block takes the
// kTcRows rows of four slices; a source's neighbours lie mostly near it in
// sorted order, so arrivals at the kTcWin ids around those rows are counted
// in LDS (a local rank per edge), and each touched id then takes one global
// atomic for the block's whole count, whose return is the base added to the
// local ranks.  Arrivals outside the window take a global atomic each.  The
// ranks of one T-row are distinct and dense (0 .. in-degree - 1) as before;
// which edge gets which rank is as unordered as with one atomic per edge.
// A local rank is below kTcRows * K (below kTcRows when no row repeats an
// id), which the 19 bits it is packed in hold.  M4 = ell_k4(K) ELL positions
// per thread, at most kTcMaxM4.
constexpr int kTcRows = 4 * kSlice;
constexpr int kTcWin = 4096;
constexpr int kTcHalo = (kTcWin - kTcRows) / 2;
constexpr int kTcMaxM4 = 32;
static_assert(kTcRows == kBlock, "one row of the block's four slices per thread");
static_assert(kTcWin <= (1 << 12) && kTcRows * kTcMaxM4 < (1 << 19), "packed window slot and local rank");

__global__ __launch_bounds__(kBlock) void k_tcount_win(int64_t N, int K, int64_t EL,
                                                       const int32_t* __restrict__ col, uint32_t* __restrict__ cnt,
                                                       uint8_t* __restrict__ rank) {
    __shared__ uint32_t c[kTcWin];
    const int M4 = ell_k4(K);
    const int64_t b = xcd_tile(blockIdx.x, gridDim.x);   // neighbouring windows on one L2
    const int64_t w0 = b * kTcRows - kTcHalo;
    const int64_t p0 = b * kTcRows * M4;   // slices 4b .. 4b + 3
    for (int t = threadIdx.x; t < kTcWin; t += kBlock) c[t] = 0u;
    __syncthreads();
    // per position: kInvalid, kFinal | global rank, or (window slot << 19) | local rank
    constexpr uint32_t kInvalid = 0xffffffffu, kFinal = 0x80000000u;
    uint32_t st[kTcMaxM4];
#pragma unroll
    for (int m = 0; m < kTcMaxM4; ++m) {
        st[m] = kInvalid;
        if (m < M4) {
            const int64_t e = p0 + threadIdx.x + (int64_t)m * kBlock;
            int64_t i = N;
            int l = K;
            if (e < EL) ell_slot(e, K, i, l);
            if (i < N && l < K) {
                const int32_t j = col[e];
                const int64_t d = (int64_t)j - w0;
                if (d >= 0 && d < kTcWin) {
                    st[m] = ((uint32_t)d << 19) | atomicAdd(&c[d], 1u);
                } else {
                    const uint32_t q = atomicAdd(&cnt[j], 1u);
                    st[m] = kFinal | (q < 255u ? q : 255u);
                }
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kTcWin; t += kBlock) {
        const uint32_t n = c[t];
        if (n > 0u) c[t] = atomicAdd(&cnt[w0 + t], n);   // n > 0 only for ids in [0, N)
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kTcMaxM4; ++m) {
        if (m < M4 && st[m] != kInvalid) {
            const int64_t e = p0 + threadIdx.x + (int64_t)m * kBlock;
            const uint32_t q = (st[m] & kFinal) ? (st[m] & 0xffu) : c[st[m] >> 19] + (st[m] & 0x7ffffu);
            rank[e] = (uint8_t)(q < 255u ? q : 255u);
        }
    }
}

// The order of one window's T-rows: keys (cap - capped in-degree, vertex)
// sorted ascending by a bitonic network in LDS; vertices past N sort last, so
// positions below N hold exactly the vertices below N.  One block per window.
__global__ __launch_bounds__(kBlock) void k_twin_order(int64_t N, uint32_t cap, const uint32_t* __restrict__ deg,
                                                       int32_t* __restrict__ trow, int32_t* __restrict__ tpos) {
    __shared__ uint32_t key[kTWin];
    const int64_t w0 = (int64_t)blockIdx.x * kTWin;
    for (int t = threadIdx.x; t < kTWin; t += kBlock) {
        const int64_t j = w0 + t;
        const uint32_t rk = j < N ? cap - min(deg[j], cap) : cap + 1u;
        key[t] = (rk << kTWinBits) | (uint32_t)t;
    }
    __syncthreads();
    for (int size = 2; size <= kTWin; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kTWin / 2; t += kBlock) {
                const int a = 2 * t - (t & (stride - 1)), b = a + stride;   // a has the stride bit clear
                const uint32_t ka = key[a], kb = key[b];
                if ((ka > kb) == ((a & size) == 0)) {
                    key[a] = kb;
                    key[b] = ka;
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < kTWin; t += kBlock) {
        const int64_t j = w0 + (key[t] & (kTWin - 1));
        if (j < N) {
            trow[w0 + t] = (int32_t)j;
            tpos[j] = (int32_t)(w0 + t);
        }
    }
}

// slice length = 64 * min(max in-degree of its 64 T-rows, cap); one wave per slice
__global__ __launch_bounds__(kBlock) void k_tslice_len(int64_t N, int64_t nslices, uint32_t cap,
                                                       const uint32_t* __restrict__ deg,
                                                       const int32_t* __restrict__ trow,
                                                       uint32_t* __restrict__ len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t d = r < N ? min(deg[trow[r]], cap) : 0u;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) d = max(d, (uint32_t)__shfl_xor((int)d, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && (r >> 6) < nslices) len[r >> 6] = d * (uint32_t)kSlice;
}

__global__ __launch_bounds__(kBlock) void k_tscatter(int64_t N, int K, int64_t EL, uint32_t cap,
                                                     const int32_t* __restrict__ col, const float* __restrict__ w,
                                                     const uint8_t* __restrict__ rank, const int32_t* __restrict__ tpos,
                                                     const uint32_t* __restrict__ soff, uint2* __restrict__ tent,
                                                     int32_t* __restrict__ ovf,
                                                     float* __restrict__ ovw, uint32_t* __restrict__ novf) {
    const int64_t e = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // nearby T-rows on one L2
    if (e >= EL) return;
    int64_t i;
    int l;
    ell_slot(e, K, i, l);
    if (i >= N || l >= K) return;
    const int64_t j = col[e];
    const uint32_t q = rank[e];
    const uint32_t o = wave_append(novf, q >= cap);
    if (q < cap) {
        const int64_t pj = tpos[j];
        const int64_t p = (int64_t)soff[pj >> 6] + (int64_t)q * kSlice + (pj & (kSlice - 1));
        tent[p] = make_uint2((uint32_t)i, __float_as_uint(w[e]));
    } else {
        ovf[2 * (int64_t)o] = (int32_t)j;
        ovf[2 * (int64_t)o + 1] = (int32_t)i;
        ovw[o] = w[e];
    }
}

// Each T-row sorted by source row (a fixed summation order), then padded with
// zero-weight self entries up to its slice's length.  C >= cap: a bitonic
// network over C register slots (unused slots hold INT_MAX); C = 0: insertion
// sort in place, for long rows.  One thread per position.
template <int C>
__global__ __launch_bounds__(kBlock) void k_tsort(int64_t N, uint32_t cap, const uint32_t* __restrict__ soff,
                                                  const uint32_t* __restrict__ deg, const int32_t* __restrict__ trow,
                                                  uint2* __restrict__ tent) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int64_t j = trow[r];
    const int64_t base = (int64_t)soff[r >> 6] + (r & (kSlice - 1));
    const uint32_t len = (soff[(r >> 6) + 1] - soff[r >> 6]) / kSlice;
    const uint32_t n = min(deg[j], cap);
    if (C > 0) {
        constexpr int CC = C > 0 ? C : 1;
        int32_t k[CC];
        float v[CC];
#pragma unroll
        for (int q = 0; q < CC; ++q) {
            const uint2 ev = (uint32_t)q < n ? tent[base + (int64_t)q * kSlice] : make_uint2(0u, 0u);
            k[q] = (uint32_t)q < n ? (int32_t)ev.x : INT32_MAX;
            v[q] = (uint32_t)q < n ? __uint_as_float(ev.y) : 0.0f;
        }
#pragma unroll
        for (int size = 2; size <= CC; size <<= 1) {
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
                for (int a = 0; a < CC; ++a) {
                    const int b2 = a ^ stride;
                    if (b2 > a) {
                        const bool up = (a & size) == 0;
                        const bool sw = up ? k[a] > k[b2] : k[a] < k[b2];
                        const int32_t tk = k[a];
                        const float tv = v[a];
                        k[a] = sw ? k[b2] : k[a];
                        v[a] = sw ? v[b2] : v[a];
                        k[b2] = sw ? tk : k[b2];
                        v[b2] = sw ? tv : v[b2];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CC; ++q) {
            if ((uint32_t)q < len) {
                tent[base + (int64_t)q * kSlice] = (uint32_t)q < n ? make_uint2((uint32_t)k[q], __float_as_uint(v[q]))
                                                                   : make_uint2((uint32_t)j, 0u);
            }
        }
        return;
    }
    for (uint32_t q = 1; q < n; ++q) {
        const uint2 ev = tent[base + (int64_t)q * kSlice];
        const int32_t sv = (int32_t)ev.x;
        uint32_t r = q;
        while (r > 0 && (int32_t)tent[base + (int64_t)(r - 1) * kSlice].x > sv) {
            tent[base + (int64_t)r * kSlice] = tent[base + (int64_t)(r - 1) * kSlice];
            --r;
        }
        tent[base + (int64_t)r * kSlice] = ev;
    }
    for (uint32_t q = n; q < len; ++q) {
        tent[base + (int64_t)q * kSlice] = make_uint2((uint32_t)j, 0u);
    }
}

// ppred[i] = position of i's predecessor (-1: none).
__global__ __launch_bounds__(kBlock) void k_tppred(int64_t N, const int32_t* __restrict__ pred,
                                                   const int32_t* __restrict__ tpos, int32_t* __restrict__ ppred) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t v = pred[i];
    ppred[i] = v >= 0 ? tpos[v] : -1;
}

// ------------------------------------------------- reverse of the output ---
// One thread per path.  o_p = e + alpha (d + in), in = sum_l w_l L_D(j_l)
// (own sample: r L_D(v0)), e the constant emission, d = d_pt or the extra
// first-vertex samples' estimate; seeds the adjoint of L_D (lam), of alpha,
// d_pt, r, and dL/dg through the extra samples.
__global__ __launch_bounds__(kBlock) void k_out_adjoint(pg_paths P, Consts c, const int32_t* __restrict__ inv,
                                                        const int32_t* __restrict__ col, const float* __restrict__ w,
                                                        const float* __restrict__ gw, const float* __restrict__ xD,
                                                        const float* __restrict__ dpt, const float* __restrict__ r,
                                                        const float* __restrict__ alpha,
                                                        const float* __restrict__ gimg, float* __restrict__ abar,
                                                        float* __restrict__ dptbar, float* __restrict__ rbar,
                                                        const int32_t* __restrict__ tpos, float* __restrict__ lam,
                                                        double* __restrict__ gpart) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gl = 0.0;
    const int64_t N = P.n_vertices;
    if (p < P.n_paths) {
        const int64_t a = P.path_offsets[p], e = P.path_offsets[p + 1];
        if (e > a && a >= 0 && e <= N) {
            const int64_t px = p / P.spp;
            const int64_t s0 = inv[a];
            const float is = 1.0f / (float)P.spp;
            const f3 ob{gimg[3 * px] * is, gimg[3 * px + 1] * is, gimg[3 * px + 2] * is};
            const float al = alpha[s0];
            const bool extra = P.n_extra > 0;
            f3 ddg{0.f, 0.f, 0.f};
            const f3 d = extra ? extra_direct(P, p, a, ld3(P.dir_in, a), c.rho, c.g, c.sun, c.env_pdf, &ddg)
                               : ld3(dpt, s0);
            const f3 zb{al * ob.x, al * ob.y, al * ob.z};
            if (extra) gl += (double)dot3(zb, ddg);
            if (c.final_gather == 0) {
                f3 in{0.f, 0.f, 0.f}, ing{0.f, 0.f, 0.f};
                for (int l = 0; l < c.K; ++l) {
                    const int64_t e = eidx(s0, l, c.K);
                    const int64_t j = col[e];
                    const float ww = w[e], gg = gw[e];
                    const f3 xv = ld3(xD, j);
                    in = f3{fmaf(ww, xv.x, in.x), fmaf(ww, xv.y, in.y), fmaf(ww, xv.z, in.z)};
                    ing = f3{fmaf(gg, xv.x, ing.x), fmaf(gg, xv.y, ing.y), fmaf(gg, xv.z, ing.z)};
                    const int64_t pj = tpos[j];
                    atomicAdd(&lam[3 * pj], ww * zb.x);
                    atomicAdd(&lam[3 * pj + 1], ww * zb.y);
                    atomicAdd(&lam[3 * pj + 2], ww * zb.z);
                }
                abar[s0] += dot3(ob, f3{d.x + in.x, d.y + in.y, d.z + in.z});
                gl += (double)dot3(zb, ing);
            } else {
                const f3 xv = ld3(xD, s0);
                const float rr = r[s0];
                abar[s0] += dot3(ob, f3{fmaf(rr, xv.x, d.x), fmaf(rr, xv.y, d.y), fmaf(rr, xv.z, d.z)});
                rbar[s0] += dot3(zb, xv);
                const int64_t ps = tpos[s0];
                atomicAdd(&lam[3 * ps], rr * zb.x);
                atomicAdd(&lam[3 * ps + 1], rr * zb.y);
                atomicAdd(&lam[3 * ps + 2], rr * zb.z);
            }
            if (!extra) {   // the extra samples replace d_pt in the output
                dptbar[3 * s0] += zb.x;
                dptbar[3 * s0 + 1] += zb.y;
                dptbar[3 * s0 + 2] += zb.z;
            }
        }
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[blockIdx.x] = t;
}

// ------------------------------------------ forward with the sums kept ---
// The two-pass aggregation of a taped render that also keeps, per row, the
// neighbour sum z_i = sum_l w_il x(j_l) and its g-derivative
// zg_i = sum_l dw_il/dg x(j_l) (z then zg, six floats) for the reverse
// sweep.  z takes the same slots and FMAs as k_spmv_c16, so y is the same bit
// for bit; zg the same as the recomputing k_rev_rows.
template <int KT, int BS>
__global__ __launch_bounds__(BS) void k_spmv_c16_tape(int64_t N, int K, const int16_t* __restrict__ c16,
                                                      const uint32_t* __restrict__ c16_base,
                                                      const int32_t* __restrict__ ovf, const float* __restrict__ w,
                                                      const float* __restrict__ gw, const float* __restrict__ x,
                                                      const float* __restrict__ b, const float* __restrict__ alpha,
                                                      float* __restrict__ y, float* __restrict__ zt, int group) {
    const int64_t tile = grouped_tile(blockIdx.x, gridDim.x, group);
    const int64_t i = tile * BS + threadIdx.x;
    if (i >= N) return;
    constexpr int NQ = KT / 4;
    const int64_t base = ell_row(i, K);
    f32x4 ww[NQ], gg[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        ww[q] = ld_quad_nt(w + base + q * kQuadStride);
        gg[q] = ld_quad_nt(gw + base + q * kQuadStride);
    }
    int32_t j[KT];
    c16_row_ids<KT>(i, K, c16, c16_base, ovf, j);
    float ax = 0.f, ay = 0.f, az = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int l = 0; l < KT; ++l) {
        const f3 xv = ld3(x, j[l]);
        const float wl = ww[l >> 2][l & 3], gl = gg[l >> 2][l & 3];
        ax = fmaf(wl, xv.x, ax);
        ay = fmaf(wl, xv.y, ay);
        az = fmaf(wl, xv.z, az);
        gx = fmaf(gl, xv.x, gx);
        gy = fmaf(gl, xv.y, gy);
        gz = fmaf(gl, xv.z, gz);
    }
    const f3 bb = ld3(b, i);
    const float a = alpha[i];
    st3_nt(y, i, f3{fmaf(a, ax, bb.x), fmaf(a, ay, bb.y), fmaf(a, az, bb.z)});
    st3_nt(zt, 2 * i, f3{ax, ay, az});
    st3_nt(zt, 2 * i + 1, f3{gx, gy, gz});
}

hipError_t launch_spmv_c16_tape(int64_t N, int K, const int16_t* c16, const uint32_t* c16_base, const int32_t* ovf,
                                const float* w, const float* gw, const float* x, const float* b, const float* alpha,
                                float* y, float* zt, hipStream_t s, int tile, int tile_group) {
    if (N == 0) return hipSuccess;
    dispatch_tile(tile, [&](auto bs) {
        constexpr int BS = decltype(bs)::value;
        switch (ell_k4(K)) {
        case 8: hipLaunchKernelGGL((k_spmv_c16_tape<8, BS>), dim3((unsigned)div_up(N, BS)), dim3(BS), 0, s, N, K, c16, c16_base, ovf, w, gw, x, b, alpha, y, zt, tile_group); break;
        case 12: hipLaunchKernelGGL((k_spmv_c16_tape<12, BS>), dim3((unsigned)div_up(N, BS)), dim3(BS), 0, s, N, K, c16, c16_base, ovf, w, gw, x, b, alpha, y, zt, tile_group); break;
        case 16: hipLaunchKernelGGL((k_spmv_c16_tape<16, BS>), dim3((unsigned)div_up(N, BS)), dim3(BS), 0, s, N, K, c16, c16_base, ovf, w, gw, x, b, alpha, y, zt, tile_group); break;
        default: break;   // not carved for other K4 (see sums_taped)
        }
    });
    return hipGetLastError();
}

// --------------------------------------------- reverse of one iteration ---
// Row i: y_i = b_i + alpha_i z_i, z_i = sum_l w_il L_{t-1}(j_l), L_t(v) = y(succ v).
// The adjoint of y_i is lam_t(pred i), read at the predecessor's position
// (ppred).  Accumulates d/d alpha_i += <ybar, z_i>
// and d/d b_i += ybar, stores zbar_i = alpha_i ybar and adds
// <zbar_i, sum_l dw_il/dg L_{t-1}(j_l)> to the block's dL/dg slot.  One thread
// per row over the sliced-ELL edges (all K loads issued before the gathers),
// as in the forward product.  KT = ell_k4(K) at compile time, 0: runtime.
template <int KT, bool C16>
__global__ __launch_bounds__(kBlock) void k_rev_rows(int64_t N, int Kr, const int32_t* __restrict__ col,
                                                     const int16_t* __restrict__ c16,
                                                     const uint32_t* __restrict__ c16_base,
                                                     const int32_t* __restrict__ c16_ovf,
                                                     const float* __restrict__ w, const float* __restrict__ gw,
                                                     const float* __restrict__ xprev, const float* __restrict__ lam,
                                                     const int32_t* __restrict__ ppred,
                                                     const float* __restrict__ alpha, float* __restrict__ abar,
                                                     float* __restrict__ bbar, float* __restrict__ zbar,
                                                     double* __restrict__ gpart) {
    const int64_t tile = blockIdx.x;   // launch order, as the forward product
    const int64_t i = tile * kBlock + threadIdx.x;
    const int K = KT ? KT : Kr;
    double gl = 0.0;
    if (i < N) {
        const int64_t base = ell_row(i, K);
        float zx = 0.f, zy = 0.f, zz = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        auto acc = [&](int32_t jl, float wl, float gl_) {
            const f3 xv = ld3(xprev, jl);
            zx = fmaf(wl, xv.x, zx);
            zy = fmaf(wl, xv.y, zy);
            zz = fmaf(wl, xv.z, zz);
            gx = fmaf(gl_, xv.x, gx);
            gy = fmaf(gl_, xv.y, gy);
            gz = fmaf(gl_, xv.z, gz);
        };
        if constexpr (C16 && KT > 0) {   // ids from the compact layout (the same ids, the same order)
            constexpr int NQ = KT / 4;
            f32x4 ww[NQ], gg[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                ww[q] = ld_quad_nt(w + base + q * kQuadStride);
                gg[q] = ld_quad_nt(gw + base + q * kQuadStride);
            }
            int32_t j[KT];
            c16_row_ids<KT>(i, K, c16, c16_base, c16_ovf, j);
#pragma unroll
            for (int l = 0; l < KT; ++l) acc(j[l], ww[l >> 2][l & 3], gg[l >> 2][l & 3]);
        } else if (KT) {
            constexpr int NQ = KT > 0 ? KT / 4 : 1;
            i32x4 j[NQ];
            f32x4 ww[NQ], gg[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                j[q] = ld_quad_nt(col + base + q * kQuadStride);
                ww[q] = ld_quad_nt(w + base + q * kQuadStride);
                gg[q] = ld_quad_nt(gw + base + q * kQuadStride);
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
                for (int c = 0; c < 4; ++c) acc(j[q][c], ww[q][c], gg[q][c]);
            }
        } else {
            for (int q = 0; 4 * q < K; ++q) {   // every slot of the last quad: the padding adds +0
                const i32x4 jq = ld_quad_nt(col + base + q * kQuadStride);
                const f32x4 wq = ld_quad_nt(w + base + q * kQuadStride);
                const f32x4 gq = ld_quad_nt(gw + base + q * kQuadStride);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc(jq[c], wq[c], gq[c]);
            }
        }
        const int64_t pv = __builtin_nontemporal_load(ppred + i);
        const f3 yb = pv >= 0 ? ld3(lam, pv) : f3{0.f, 0.f, 0.f};
        abar[i] += dot3(yb, f3{zx, zy, zz});
        bbar[3 * i] += yb.x;
        bbar[3 * i + 1] += yb.y;
        bbar[3 * i + 2] += yb.z;
        const float al = alpha[i];
        const f3 zb{al * yb.x, al * yb.y, al * yb.z};
        st3_nt(zbar, i, zb);
        gl = (double)dot3(zb, f3{gx, gy, gz});
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[tile] += t;
}

// k_rev_rows with z_i and zg_i read from the forward's tape (zt: six floats
// per row) instead of gathered again: the same values, the same updates and
// the same block partials, so the same results bit for bit.
__global__ __launch_bounds__(kBlock) void k_rev_rows_taped(int64_t N, const float* __restrict__ zt,
                                                           const float* __restrict__ lam,
                                                           const int32_t* __restrict__ ppred,
                                                           const float* __restrict__ alpha, float* __restrict__ abar,
                                                           float* __restrict__ bbar, float* __restrict__ zbar,
                                                           double* __restrict__ gpart) {
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);   // the predecessors' lambda lines on one L2
    const int64_t i = tile * kBlock + threadIdx.x;
    double gl = 0.0;
    if (i < N) {
        const f3 z = ld3(zt, 2 * i), zg = ld3(zt, 2 * i + 1);
        const int64_t pv = __builtin_nontemporal_load(ppred + i);
        const f3 yb = pv >= 0 ? ld3(lam, pv) : f3{0.f, 0.f, 0.f};
        abar[i] += dot3(yb, z);
        bbar[3 * i] += yb.x;
        bbar[3 * i + 1] += yb.y;
        bbar[3 * i + 2] += yb.z;
        const float al = alpha[i];
        const f3 zb{al * yb.x, al * yb.y, al * yb.z};
        st3_nt(zbar, i, zb);
        gl = (double)dot3(zb, zg);
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[tile] += t;
}

// lam_{t-1}(j) = sum over rows i with j in N(i) of w_ij zbar_i, stored at j's
// position r: one thread per position over the sliced-ELL transpose (every
// lane of a wave runs its slice's length, the zero-weight padding included: a
// per-lane bound measured slower), eight entries loaded ahead (four: 7% slower).
__global__ __launch_bounds__(kBlock) void k_rev_cols(int64_t N, const uint32_t* __restrict__ soff,
                                                     const uint2* __restrict__ tent,
                                                     const float* __restrict__ zbar, float* __restrict__ lam) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int64_t base = (int64_t)soff[r >> 6] + (r & (kSlice - 1));
    const uint32_t len = (soff[(r >> 6) + 1] - soff[r >> 6]) / kSlice;
    float ax = 0.f, ay = 0.f, az = 0.f;
    uint32_t q = 0;
    auto block = [&](auto n) {   // n entries: all ids and weights loaded, then the gathers in order
        constexpr int U = decltype(n)::value;
        int32_t src[U];
        float ww[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t ev = __builtin_nontemporal_load(
                reinterpret_cast<const uint64_t*>(tent) + base + (int64_t)(q + u) * kSlice);
            src[u] = (int32_t)(uint32_t)ev;
            ww[u] = __uint_as_float((uint32_t)(ev >> 32));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const f3 zb = ld3(zbar, src[u]);
            ax = fmaf(ww[u], zb.x, ax);
            ay = fmaf(ww[u], zb.y, ay);
            az = fmaf(ww[u], zb.z, az);
        }
        q += U;
    };
    while (q + 8 <= len) block(std::integral_constant<int, 8>{});
    if (q + 4 <= len) block(std::integral_constant<int, 4>{});
    for (; q < len; ++q) {
        const uint2 ev = tent[base + (int64_t)q * kSlice];
        const f3 zb = ld3(zbar, (int32_t)ev.x);
        const float ww = __uint_as_float(ev.y);
        ax = fmaf(ww, zb.x, ax);
        ay = fmaf(ww, zb.y, ay);
        az = fmaf(ww, zb.z, az);
    }
    st3_nt(lam, r, f3{ax, ay, az});
}

__global__ __launch_bounds__(kBlock) void k_rev_overflow(const int32_t* __restrict__ ovf, const float* __restrict__ ovw,
                                                         const uint32_t* __restrict__ novf,
                                                         const int32_t* __restrict__ tpos,
                                                         const float* __restrict__ zbar, float* __restrict__ lam) {
    const uint32_t n = *novf;
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x) {
        const int64_t j = tpos[ovf[2 * (int64_t)o]], i = ovf[2 * (int64_t)o + 1];
        const float ww = ovw[o];
        const f3 zb = ld3(zbar, i);
        atomicAdd(&lam[3 * j], ww * zb.x);
        atomicAdd(&lam[3 * j + 1], ww * zb.y);
        atomicAdd(&lam[3 * j + 2], ww * zb.z);
    }
}

// ------------------------------- reverse of the path-traced initial value ---
// L_0(v) = alpha_u (d_pt_u + r_u L_0(u)), u = succ v.  Its adjoint runs from
// each path's first vertex: lam_0(u) += alpha_u r_u lam_0(v), v = pred u, an
// affine recurrence l(u) = A_u + B_u l(v) with A_u the adjoint the sweep left
// at u and B_u = alpha_u r_u (B = 0 at the first vertex).  One wave per path
// takes 64 vertices at a time: a wave-level inclusive scan composes the
// lanes' maps (G2 o G1 = (A2 + B2 A1, B2 B1)), applied to the value carried
// from the previous chunk; each lane then adds its vertex's albedo, d_pt and r
// adjoints from its predecessor's l and stores its own l (lam held at the
// T-row positions tpos; null: at the vertices).
__global__ __launch_bounds__(kBlock) void k_pt_adjoint(int64_t P, int64_t N, const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ inv,
                                                       const float* __restrict__ alpha, const float* __restrict__ dpt,
                                                       const float* __restrict__ r, const float* __restrict__ x0,
                                                       const int32_t* __restrict__ tpos,
                                                       float* __restrict__ lam, float* __restrict__ abar,
                                                       float* __restrict__ dptbar, float* __restrict__ rbar) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;   // uniform over the wave
    if (p >= P) return;
    const int64_t a = off[p], e = off[p + 1];
    if (a < 0 || e < a || e > N) return;
    f3 carry{0.f, 0.f, 0.f};   // l at the vertex before the chunk
    for (int64_t lo = a; lo < e; lo += kWave) {
        const int64_t v = lo + lane;
        const bool valid = v < e, step = valid && v > a;
        int64_t u = 0, pu = 0;
        float al = 0.0f, rr = 0.0f, B = 1.0f;   // identity past the path's end
        f3 A{0.f, 0.f, 0.f}, d{0.f, 0.f, 0.f}, xu{0.f, 0.f, 0.f};
        if (valid) {
            u = inv[v];
            pu = tpos ? tpos[u] : u;
            A = ld3(lam, pu);
            B = 0.0f;
            if (step) {
                al = alpha[u];
                rr = r[u];
                d = ld3(dpt, u);
                xu = ld3(x0, u);
                B = al * rr;
            }
        }
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const float Bo = __shfl_up(B, o, kWave);
            const float Ax = __shfl_up(A.x, o, kWave), Ay = __shfl_up(A.y, o, kWave), Az = __shfl_up(A.z, o, kWave);
            if (lane >= o) {
                A = f3{fmaf(B, Ax, A.x), fmaf(B, Ay, A.y), fmaf(B, Az, A.z)};
                B *= Bo;
            }
        }
        // l at the predecessor: the lanes below this one applied to the
        // carry (every lane shuffles; lane 0 then takes the identity)
        const float Bsh = __shfl_up(B, 1, kWave);
        const float Aex = __shfl_up(A.x, 1, kWave), Aey = __shfl_up(A.y, 1, kWave), Aez = __shfl_up(A.z, 1, kWave);
        const float Be = lane > 0 ? Bsh : 1.0f;
        const f3 Ae = lane > 0 ? f3{Aex, Aey, Aez} : f3{0.f, 0.f, 0.f};
        const f3 l{fmaf(Be, carry.x, Ae.x), fmaf(Be, carry.y, Ae.y), fmaf(Be, carry.z, Ae.z)};
        if (step) {
            abar[u] += dot3(l, f3{fmaf(rr, xu.x, d.x), fmaf(rr, xu.y, d.y), fmaf(rr, xu.z, d.z)});
            dptbar[3 * u] += al * l.x;
            dptbar[3 * u + 1] += al * l.y;
            dptbar[3 * u + 2] += al * l.z;
            rbar[u] += al * dot3(l, xu);
            st3(lam, pu, f3{fmaf(B, carry.x, A.x), fmaf(B, carry.y, A.y), fmaf(B, carry.z, A.z)});
        }
        const float Bl = __shfl(B, kWave - 1, kWave);
        const f3 Al{__shfl(A.x, kWave - 1, kWave), __shfl(A.y, kWave - 1, kWave), __shfl(A.z, kWave - 1, kWave)};
        carry = f3{fmaf(Bl, carry.x, Al.x), fmaf(Bl, carry.y, Al.y), fmaf(Bl, carry.z, Al.z)};
    }
}

// ----------------------------------------- reverse of the direct terms ---
// Mirrors k_edges: recomputes the weights, then
//   d/d alpha_i += <bbar_i, d_agg_i>,
//   dL/dg += <alpha_i bbar_i, d d_agg_i/dg> + <d_pt bar_i, d d_pt_i/dg> + rbar_i r_i h(u_w,i).
template <int KP>
__global__ __launch_bounds__(kBlock) void k_edges_adjoint(int64_t N, Consts c, const int32_t* __restrict__ col,
                                                          const VRec* __restrict__ rec,
                                                          const float* __restrict__ bbar,
                                                          const float* __restrict__ dptbar,
                                                          const float* __restrict__ rbar, float* __restrict__ abar,
                                                          double* __restrict__ gpart, const int32_t* __restrict__ perm,
                                                          const float* __restrict__ dir_pl,
                                                          const float* __restrict__ l_pl) {
    constexpr int GR = kBlock / KP;
    __shared__ f3 tsh[GR][KP];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % KP, grp = threadIdx.x / KP;
    const int64_t i = tile * GR + grp;
    const int K = c.K;
    const bool act = i < N && lane < K;
    f3 t{0.f, 0.f, 0.f}, w{0.f, 0.f, 0.f}, we{0.f, 0.f, 0.f}, ls{0.f, 0.f, 0.f}, le{0.f, 0.f, 0.f},
        lp{0.f, 0.f, 0.f};
    float alpha = 0.0f;
    f3 dpl{0.f, 0.f, 0.f}, lpl{0.f, 0.f, 0.f};
    if (act) {
        const int32_t jn = col[eidx(i, lane, K)];
        if (dir_pl) {
            dpl = ld3(dir_pl, perm[jn]);
            lpl = ld3(l_pl, perm[jn]);
        }
        const float4* r4 = reinterpret_cast<const float4*>(rec + jn);
        float4 a0 = r4[0], a1 = r4[1], a2 = r4[2], a3 = r4[3], a4 = r4[4];
        t = f3{a0.x, a0.y, a0.z};
        w = f3{a0.w, a1.x, a1.y};
        we = f3{a1.z, a1.w, a2.x};
        ls = f3{a2.y, a2.z, a2.w};
        le = f3{a3.x, a3.y, a3.z};
        lp = f3{a3.w, a4.x, a4.y};
        alpha = a4.z;
    }
    tsh[grp][lane] = t;
    __syncthreads();
    const f3 ti = tsh[grp][0];
    float mplus = 0.0f, menv = 0.0f;
    for (int l = 0; l < K; ++l) {
        const f3 tl = tsh[grp][l];
        mplus += c.pdf(one_minus_cos(tl, w));
        menv += c.pdf(one_minus_cos(tl, we));
    }
    const float Kpe = (float)K * c.env_pdf;
    const float u_w = one_minus_cos(ti, w), u_e = one_minus_cos(ti, we);
    const float rho = c.rho(u_w), rho_e = c.rho(u_e);
    const float wp = rho / (mplus + Kpe), wev = rho_e / (menv + Kpe);
    const float hw = hg_dlog(c.g, u_w), he = hg_dlog(c.g, u_e);
    // value and g-derivative of each record's contribution
    float cx = act ? wev * le.x + wp * lp.x : 0.f, cy = act ? wev * le.y + wp * lp.y : 0.f,
          cz = act ? wev * le.z + wp * lp.z : 0.f;
    float hx = act ? wev * he * le.x + wp * hw * lp.x : 0.f, hy = act ? wev * he * le.y + wp * hw * lp.y : 0.f,
          hz = act ? wev * he * le.z + wp * hw * lp.z : 0.f;
    float sx = act ? ls.x : 0.f, sy = act ? ls.y : 0.f, sz = act ? ls.z : 0.f;
    cx = group_sum<KP>(cx);
    cy = group_sum<KP>(cy);
    cz = group_sum<KP>(cz);
    hx = group_sum<KP>(hx);
    hy = group_sum<KP>(hy);
    hz = group_sum<KP>(hz);
    sx = group_sum<KP>(sx);
    sy = group_sum<KP>(sy);
    sz = group_sum<KP>(sz);
    // point light: value and g-derivative of the neighbours' delta samples
    float rpl = 0.f, hpl = 0.f;
    if (act && dir_pl) {
        const float u = one_minus_cos(ti, dpl);
        rpl = c.rho(u);
        hpl = rpl * hg_dlog(c.g, u);
    }
    float qx = rpl * lpl.x, qy = rpl * lpl.y, qz = rpl * lpl.z;
    float gx = hpl * lpl.x, gy = hpl * lpl.y, gz = hpl * lpl.z;
    if (dir_pl) {
        qx = group_sum<KP>(qx);
        qy = group_sum<KP>(qy);
        qz = group_sum<KP>(qz);
        gx = group_sum<KP>(gx);
        gy = group_sum<KP>(gy);
        gz = group_sum<KP>(gz);
    }
    double gl = 0.0;
    if (i < N && lane == 0) {
        const float u_s = one_minus_cos(ti, c.sun);
        const float rho_sun = c.rho(u_s), hs = hg_dlog(c.g, u_s);
        const float invK = 1.0f / (float)K;
        f3 dagg{fmaf(rho_sun * invK, sx, cx), fmaf(rho_sun * invK, sy, cy), fmaf(rho_sun * invK, sz, cz)};
        if (dir_pl) dagg = f3{fmaf(invK, qx, dagg.x), fmaf(invK, qy, dagg.y), fmaf(invK, qz, dagg.z)};
        const f3 bb = ld3(bbar, i);
        abar[i] += dot3(bb, dagg);
        const f3 db{alpha * bb.x, alpha * bb.y, alpha * bb.z};
        const float ks = rho_sun * hs * invK;
        gl += (double)dot3(db, f3{fmaf(ks, sx, hx), fmaf(ks, sy, hy), fmaf(ks, sz, hz)});
        if (dir_pl) gl += (double)(invK * dot3(db, f3{gx, gy, gz}));
        // own direct term and continuation ratio
        const float p_w = c.pdf(u_w), p_e = c.pdf(u_e);
        const float f_env = rho_e / (p_e + c.env_pdf), f_out = rho / (p_w + c.env_pdf);
        const f3 pb = ld3(dptbar, i);
        const f3 dd{rho_sun * hs * ls.x + f_env * he * le.x + f_out * hw * lp.x,
                    rho_sun * hs * ls.y + f_env * he * le.y + f_out * hw * lp.y,
                    rho_sun * hs * ls.z + f_env * he * le.z + f_out * hw * lp.z};
        gl += (double)dot3(pb, dd);
        if (dir_pl) gl += (double)(hpl * dot3(pb, lpl));   // lane 0: the receiver's own sample
        gl += (double)(rbar[i] * (rho / p_w) * hw);
    }
    const double tsum = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[tile] = tsum;
}

// ------------------------------------------- albedo grid and per vertex ---
// The 256 vertices of a block are consecutive in the spatial order, so their
// 8 x 256 trilinear contributions fall on a few dozen voxels: they are summed
// in an LDS hash table (open addressing on the voxel index) and each distinct
// voxel is added to the grid once.  A contribution that finds no free slot
// within kProbe probes goes to the grid directly.
constexpr int kHash = 1024;
constexpr int kProbe = 32;
constexpr uint32_t kEmpty = 0xffffffffu;

__global__ __launch_bounds__(kBlock) void k_grid_adjoint(int64_t N, pg_paths P, const int32_t* __restrict__ perm,
                                                         const float* __restrict__ abar,
                                                         float* __restrict__ grad_grid,
                                                         float* __restrict__ grad_alpha) {
    __shared__ uint32_t hkey[kHash];
    __shared__ float hval[kHash];
    for (int h = threadIdx.x; h < kHash; h += kBlock) {
        hkey[h] = kEmpty;
        hval[h] = 0.0f;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool grid = grad_grid && P.albedo_grid;
    if (i < N) {
        const int64_t v = perm[i];
        const float ab = abar[i];
        if (grad_alpha) grad_alpha[v] = ab;
        if (grid) {
            uint32_t idx[8];
            float tw[8];
            trilerp_corners(P.albedo_grid_res, P.pos[3 * v], P.pos[3 * v + 1], P.pos[3 * v + 2], idx, tw);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (tw[q] == 0.0f) continue;
                const float val = ab * tw[q];
                uint32_t h = (idx[q] * 2654435761u) >> 22;   // 10-bit multiplicative hash
                bool done = false;
                for (int probe = 0; probe < kProbe && !done; ++probe, h = (h + 1) & (kHash - 1)) {
                    const uint32_t k = atomicCAS(&hkey[h], kEmpty, idx[q]);
                    if (k == kEmpty || k == idx[q]) {
                        atomicAdd(&hval[h], val);
                        done = true;
                    }
                }
                if (!done) atomicAdd(&grad_grid[idx[q]], val);
            }
        }
    }
    __syncthreads();
    if (grid)
        for (int h = threadIdx.x; h < kHash; h += kBlock)
            if (hkey[h] != kEmpty) atomicAdd(&grad_grid[hkey[h]], hval[h]);
}

// dL/dg = the sum of the fixed slots, in two fixed-order levels: each block
// sums one chunk of kReduceChunk slots, then one block sums the chunk totals
// (out_f == NULL: write the block totals to out_d instead).
constexpr int kReduceChunk = 4096;
__global__ __launch_bounds__(kBlock) void k_reduce_g(int64_t n, const double* __restrict__ gpart,
                                                     double* __restrict__ out_d, float* __restrict__ out_f) {
    const int64_t lo = out_f ? 0 : (int64_t)blockIdx.x * kReduceChunk;
    const int64_t hi = out_f ? n : (lo + kReduceChunk < n ? lo + kReduceChunk : n);
    double v = 0.0;
    for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) v += gpart[q];
    const double t = block_sum_d(v);
    if (threadIdx.x == 0) {
        if (out_f) out_f[0] = (float)t;
        else out_d[blockIdx.x] = t;
    }
}

// ----------------------------------------------------------------- host ---

void carve_back(Carver& cv, BackBufs& bb, const RenderBufs& r, const pg_paths* p) {
    const int64_t N = r.N, E = N * (int64_t)r.K;
    if (r.clusters) {   // no transpose: the cluster's member range serves both products
        bb.n_rows = div_up(N > 0 ? N : 1, kBlock);
        bb.n_edge = div_up(N > 0 ? N : 1, kBlock);
        bb.n_out = div_up(r.P > 0 ? r.P : 1, kBlock);
        bb.n_slots = bb.n_rows + bb.n_edge + bb.n_out;
        bb.lam_a = cv.take<float>(3 * N);
        bb.lam_b = cv.take<float>(3 * N);
        bb.zbar = cv.take<float>(3 * N);
        bb.abar = cv.take<float>(N);
        bb.bbar = cv.take<float>(3 * N);
        bb.dptbar = cv.take<float>(3 * N);
        bb.rbar = cv.take<float>(N);
        bb.cpid = cv.take<int32_t>(N);
        bb.gpart = cv.take<double>(bb.n_slots);
        bb.gchunk = cv.take<double>(div_up(bb.n_slots, kReduceChunk));
        bb.image = cv.take<float>((int64_t)p->width * p->height * 3);
        return;
    }
    int kp = 1;
    while (kp < (r.K > 0 ? r.K : 1)) kp *= 2;
    bb.n_rows = div_up(N > 0 ? N : 1, kBlock);          // reverse sweep: one thread per row
    bb.n_edge = div_up(N > 0 ? N : 1, kBlock / kp);     // direct-term adjoint: KP lanes per row
    bb.n_out = div_up(r.P > 0 ? r.P : 1, kBlock);
    bb.n_slots = bb.n_rows + bb.n_edge + bb.n_out;
    bb.lam_a = cv.take<float>(3 * N);
    bb.lam_b = cv.take<float>(3 * N);
    bb.zbar = cv.take<float>(3 * N);
    bb.abar = cv.take<float>(N);
    bb.bbar = cv.take<float>(3 * N);
    bb.dptbar = cv.take<float>(3 * N);
    bb.rbar = cv.take<float>(N);
    bb.cap = (uint32_t)(2 * (r.K > 0 ? r.K : 1));
    bb.nslices = div_up(N > 0 ? N : 1, kSlice);
    bb.tdeg = cv.take<uint32_t>(N + 1);
    bb.tlen = cv.take<uint32_t>(bb.nslices + 1);
    bb.trank = cv.take<uint8_t>(ell_size(N, r.K));
    bb.soff = cv.take<uint32_t>(bb.nslices + 1);
    bb.trow = cv.take<int32_t>(div_up(N > 0 ? N : 1, kTWin) * kTWin);
    bb.tpos = cv.take<int32_t>(N > 0 ? N : 1);
    bb.ppred = cv.take<int32_t>(N > 0 ? N : 1);
    bb.tpart = cv.take<uint32_t>(scan_partials_bytes(bb.nslices + 1) / 4);
    bb.tent = cv.take<uint2>(bb.nslices * kSlice * (int64_t)bb.cap);
    bb.ovf = cv.take<int32_t>(2 * E);
    bb.ovw = cv.take<float>(E);
    bb.novf = cv.take<uint32_t>(64);
    bb.gpart = cv.take<double>(bb.n_slots);
    bb.gchunk = cv.take<double>(div_up(bb.n_slots, kReduceChunk));
    bb.image = cv.take<float>((int64_t)p->width * p->height * 3);
}

#define PG_TRY(x)                        \
    do {                                 \
        hipError_t e_ = (x);             \
        if (e_ != hipSuccess) return e_; \
    } while (0)

// The reverse mode of the cluster relation: the same steps in cluster order,
// with the transposed product taken over each sample's cluster.
static hipError_t run_backward_clusters(const pg_paths* p, const pg_params* q, RenderBufs& r, BackBufs& bb,
                                        const float* gimg, float* grad_grid, float* grad_alpha, float* grad_g,
                                        hipStream_t s) {
    const int64_t N = r.N;
    const int D = r.D;
    const Consts c = make_consts(q, r.K);
    PG_TRY(launch_fill(bb.lam_a, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.abar, (size_t)N * 4, s));
    PG_TRY(launch_fill(bb.bbar, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.dptbar, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.rbar, (size_t)N * 4, s));
    PG_TRY(launch_fill(bb.gpart, (size_t)bb.n_slots * 8, s));
    if (grad_grid && p->albedo_grid) {
        const int64_t R = p->albedo_grid_res;
        PG_TRY(launch_fill(grad_grid, (size_t)(R * R * R) * 4, s));
    }
    PG_TRY(launch_cluster_cpid(N, r, bb.cpid, s));
    double* g_rows = bb.gpart;
    double* g_edges = bb.gpart + bb.n_rows;
    double* g_out = bb.gpart + bb.n_rows + bb.n_edge;
    {
        ProfScope ps(s, "out_adjoint");
        PG_TRY(launch_cluster_out_adjoint(*p, c, r, gimg, bb.abar, bb.dptbar, bb.rbar, bb.lam_a, g_out, bb.n_out, s));
    }
    float* lam = bb.lam_a;
    float* lam_prev = bb.lam_b;
    for (int t = D; t >= 1 && N > 0; --t) {
        PG_TRY(launch_cluster_reverse_step(r, q, t, lam, lam_prev, bb.abar, bb.bbar, bb.zbar, g_rows, s));
        std::swap(lam, lam_prev);
    }
    if (q->init == PG_INIT_PT && N > 0) {
        ProfScope ps(s, "pt_adjoint");
        hipLaunchKernelGGL(k_pt_adjoint, dim3((unsigned)div_up((r.P > 0 ? r.P : 1) * kWave, kBlock)), dim3(kBlock), 0, s,
                           r.P, N, p->path_offsets, r.cl.cinv, r.alpha, r.dpt, r.r, r.traj, (const int32_t*)nullptr,
                           lam, bb.abar, bb.dptbar, bb.rbar);
        PG_TRY(hipGetLastError());
    }
    {
        ProfScope ps(s, "edges_adjoint");
        PG_TRY(launch_cluster_edges_adjoint(*p, c, r, bb.cpid, bb.bbar, bb.dptbar, bb.rbar, bb.abar, g_edges, s));
    }
    if (N > 0) {
        ProfScope ps(s, "grid_adjoint");
        hipLaunchKernelGGL(k_grid_adjoint, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, *p, bb.cpid,
                           bb.abar, grad_grid, grad_alpha);
        PG_TRY(hipGetLastError());
    }
    if (grad_g) {
        const int64_t nchunk = div_up(bb.n_slots, kReduceChunk);
        hipLaunchKernelGGL(k_reduce_g, dim3((unsigned)nchunk), dim3(kBlock), 0, s, bb.n_slots, bb.gpart, bb.gchunk,
                           (float*)nullptr);
        hipLaunchKernelGGL(k_reduce_g, dim3(1), dim3(kBlock), 0, s, nchunk, (const double*)bb.gchunk,
                           (double*)nullptr, grad_g);
        PG_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t run_backward(const pg_paths* p, const pg_params* q, RenderBufs& r, BackBufs& bb, const float* gimg,
                        float* grad_grid, float* grad_alpha, float* grad_g, hipStream_t s) {
    if (r.clusters) return run_backward_clusters(p, q, r, bb, gimg, grad_grid, grad_alpha, grad_g, s);
    const int64_t N = r.N, E = N * (int64_t)r.K;
    const int K = r.K, D = r.D;
    const Consts c = make_consts(q, K);
    PG_TRY(launch_fill(bb.lam_a, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.abar, (size_t)N * 4, s));
    PG_TRY(launch_fill(bb.bbar, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.dptbar, (size_t)N * 12, s));
    PG_TRY(launch_fill(bb.rbar, (size_t)N * 4, s));
    PG_TRY(launch_fill(bb.gpart, (size_t)bb.n_slots * 8, s));
    if (grad_grid && p->albedo_grid) {
        const int64_t R = p->albedo_grid_res;
        PG_TRY(launch_fill(grad_grid, (size_t)(R * R * R) * 4, s));
    }
    if (N > 0) {
        // sliced-ELL transpose of W (sorted ids)
        ProfScope ps(s, "transpose");
        PG_TRY(launch_fill(bb.tdeg, (size_t)(N + 1) * 4, s));
        PG_TRY(launch_fill(bb.tlen, (size_t)(bb.nslices + 1) * 4, s));
        PG_TRY(launch_fill(bb.novf, 4, s));
        const int64_t EL = ell_size(N, K);
        if (ell_k4(K) <= kTcMaxM4)
            hipLaunchKernelGGL(k_tcount_win, dim3((unsigned)div_up(N, kTcRows)), dim3(kBlock), 0, s, N, K, EL, r.col,
                               bb.tdeg, bb.trank);
        else
            hipLaunchKernelGGL(k_tcount, dim3((unsigned)div_up(EL, kBlock)), dim3(kBlock), 0, s, N, K, EL, r.col,
                               bb.tdeg, bb.trank);
        hipLaunchKernelGGL(k_twin_order, dim3((unsigned)div_up(N, kTWin)), dim3(kBlock), 0, s, N, bb.cap, bb.tdeg,
                           bb.trow, bb.tpos);
        hipLaunchKernelGGL(k_tslice_len, dim3((unsigned)div_up(bb.nslices * kSlice, kBlock)), dim3(kBlock), 0, s,
                           N, bb.nslices, bb.cap, bb.tdeg, bb.trow, bb.tlen);
        PG_TRY(launch_scan_exclusive(bb.tlen, bb.soff, bb.nslices, bb.tpart, s));
        hipLaunchKernelGGL(k_tscatter, dim3((unsigned)div_up(EL, kBlock)), dim3(kBlock), 0, s, N, K, EL, bb.cap,
                           r.col, r.w, bb.trank, bb.tpos, bb.soff, bb.tent, bb.ovf, bb.ovw, bb.novf);
        auto sort = [&](auto c) {
            constexpr int C = decltype(c)::value;
            hipLaunchKernelGGL(k_tsort<C>, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, bb.cap,
                               (const uint32_t*)bb.soff, (const uint32_t*)bb.tdeg, (const int32_t*)bb.trow,
                               bb.tent);
        };
        if (bb.cap <= 8) sort(std::integral_constant<int, 8>{});
        else if (bb.cap <= 16) sort(std::integral_constant<int, 16>{});
        else if (bb.cap <= 32) sort(std::integral_constant<int, 32>{});
        else sort(std::integral_constant<int, 0>{});
        hipLaunchKernelGGL(k_tppred, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, r.pred,
                           (const int32_t*)bb.tpos, bb.ppred);
        PG_TRY(hipGetLastError());
    }
    const float* xD = r.traj + (size_t)D * N * 3;
    double* g_rows = bb.gpart;
    double* g_edges = bb.gpart + bb.n_rows;
    double* g_out = bb.gpart + bb.n_rows + bb.n_edge;
    {
        ProfScope ps(s, "out_adjoint");
        hipLaunchKernelGGL(k_out_adjoint, dim3((unsigned)bb.n_out), dim3(kBlock), 0, s, *p, c, r.g.inv, r.col, r.w,
                           r.gw, xD, r.dpt, r.r, r.alpha, gimg, bb.abar, bb.dptbar, bb.rbar, bb.tpos, bb.lam_a, g_out);
        PG_TRY(hipGetLastError());
    }
    float* lam = bb.lam_a;
    float* lam_next = bb.lam_b;
    for (int t = D; t >= 1 && N > 0; --t) {
        const float* xprev = r.traj + (size_t)(t - 1) * N * 3;
        if (r.zt) {
            ProfScope ps(s, "rev_rows");
            hipLaunchKernelGGL(k_rev_rows_taped, dim3((unsigned)bb.n_rows), dim3(kBlock), 0, s, N,
                               (const float*)(r.zt + (size_t)(t - 1) * N * 6), (const float*)lam,
                               (const int32_t*)bb.ppred, (const float*)r.alpha, bb.abar, bb.bbar, bb.zbar, g_rows);
        } else {
            ProfScope ps(s, "rev_rows");
            auto go = [&](auto kt) {
                constexpr int KT = decltype(kt)::value;
                if (KT > 0 && r.c16)
                    hipLaunchKernelGGL((k_rev_rows<KT, true>), dim3((unsigned)bb.n_rows), dim3(kBlock), 0, s, N, K,
                                       r.col, r.c16, r.c16_base, r.c16_ovf, r.w, r.gw, xprev, lam, bb.ppred, r.alpha,
                                       bb.abar, bb.bbar, bb.zbar, g_rows);
                else
                    hipLaunchKernelGGL((k_rev_rows<KT, false>), dim3((unsigned)bb.n_rows), dim3(kBlock), 0, s, N, K,
                                       r.col, r.c16, r.c16_base, r.c16_ovf, r.w, r.gw, xprev, lam, bb.ppred, r.alpha,
                                       bb.abar, bb.bbar, bb.zbar, g_rows);
            };
            switch (ell_k4(K)) {
            case 8: go(std::integral_constant<int, 8>{}); break;
            case 12: go(std::integral_constant<int, 12>{}); break;
            case 16: go(std::integral_constant<int, 16>{}); break;
            default: go(std::integral_constant<int, 0>{}); break;
            }
        }
        {
            ProfScope ps(s, "rev_cols");
            hipLaunchKernelGGL(k_rev_cols, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, bb.soff,
                               (const uint2*)bb.tent, bb.zbar, lam_next);
            hipLaunchKernelGGL(k_rev_overflow, dim3(64), dim3(kBlock), 0, s, bb.ovf, bb.ovw, bb.novf, bb.tpos,
                               bb.zbar, lam_next);
        }
        PG_TRY(hipGetLastError());
        float* tmp = lam;
        lam = lam_next;
        lam_next = tmp;
    }
    if (q->init == PG_INIT_PT && N > 0) {
        ProfScope ps(s, "pt_adjoint");
        hipLaunchKernelGGL(k_pt_adjoint, dim3((unsigned)div_up((r.P > 0 ? r.P : 1) * kWave, kBlock)), dim3(kBlock), 0, s,
                           r.P, N, p->path_offsets, r.g.inv, r.alpha, r.dpt, r.r, r.traj, (const int32_t*)bb.tpos,
                           lam, bb.abar, bb.dptbar, bb.rbar);
        PG_TRY(hipGetLastError());
    }
    if (N > 0) {
        ProfScope ps(s, "edges_adjoint");
        dispatch_kp(K, [&](auto kp) {
            constexpr int KP = decltype(kp)::value;
            hipLaunchKernelGGL(k_edges_adjoint<KP>, dim3((unsigned)div_up(N, kBlock / KP)), dim3(kBlock), 0, s, N,
                               c, r.col, r.rec, bb.bbar, bb.dptbar, bb.rbar, bb.abar, g_edges, r.g.perm, p->dir_pl,
                               p->l_pl);
        });
        PG_TRY(hipGetLastError());
    }
    if (N > 0) {
        ProfScope ps(s, "grid_adjoint");
        hipLaunchKernelGGL(k_grid_adjoint, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, *p, r.g.perm,
                           bb.abar, grad_grid, grad_alpha);
        PG_TRY(hipGetLastError());
    }
    if (grad_g) {
        const int64_t nchunk = div_up(bb.n_slots, kReduceChunk);
        hipLaunchKernelGGL(k_reduce_g, dim3((unsigned)nchunk), dim3(kBlock), 0, s, bb.n_slots, bb.gpart, bb.gchunk,
                           (float*)nullptr);
        hipLaunchKernelGGL(k_reduce_g, dim3(1), dim3(kBlock), 0, s, nchunk, (const double*)bb.gchunk,
                           (double*)nullptr, grad_g);
        PG_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pg

using namespace pg;

static void carve_all(Carver& cv, RenderBufs& r, BackBufs& bb, const pg_paths* p, const pg_params* q) {
    pg_params qt = *q;
    qt.flags |= PG_FLAG_TAPE;
    carve_render(cv, r, p, &qt);
    carve_back(cv, bb, r, p);
}

extern "C" {

pg_status pg_backward_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params))) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    if ((st = validate_clusters(paths, params))) return st;
    Carver cv(nullptr);
    RenderBufs r;
    BackBufs bb;
    carve_all(cv, r, bb, paths, params);
    *bytes = cv.size();
    return PG_OK;
}

pg_status pg_backward(const pg_paths* paths, const pg_params* params, const float* grad_image, float* grad_grid,
                      float* grad_albedo, float* grad_g, void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params))) return st;
    if (!grad_image) return fail(PG_ERR_ARG, "grad_image is NULL");
    if ((st = validate_clusters(paths, params))) return st;
    if (grad_grid && !paths->albedo_grid) return fail(PG_ERR_ARG, "grad_grid needs paths->albedo_grid");
    if (!grad_grid && !grad_albedo && !grad_g) return fail(PG_ERR_ARG, "no gradient requested");
    if (!(params->flags & PG_FLAG_CLUSTERS)) {
        const int64_t N = paths->n_vertices, K = N < params->k ? N : params->k;
        if (N * K >= ((int64_t)1 << 32) || div_up(N, kSlice) * kSlice * 2 * K >= ((int64_t)1 << 32))
            return fail(PG_ERR_UNSUPPORTED, "pg_backward needs N*K < 2^31 edges");
    }
    Carver dry(nullptr);
    RenderBufs r;
    BackBufs bb;
    carve_all(dry, r, bb, paths, params);
    if ((st = check_ws(ws, ws_bytes, dry.size()))) return st;
    Carver cv(ws);
    carve_all(cv, r, bb, paths, params);
    hipStream_t s = (hipStream_t)stream;
    pg_params qt = *params;
    qt.flags |= PG_FLAG_TAPE;
    hipError_t e;
    if (!(params->flags & PG_FLAG_TAPE)) {
        e = run_render(paths, &qt, r, nullptr, bb.image, s);
        if (e != hipSuccess) return hip_fail(e, "forward");
    }
    e = run_backward(paths, &qt, r, bb, grad_image, grad_grid, grad_albedo, grad_g, s);
    if (e != hipSuccess) return hip_fail(e, "backward");
    return finish(s, params, r.g.flag, params->flags);
}

}  // extern "C"
