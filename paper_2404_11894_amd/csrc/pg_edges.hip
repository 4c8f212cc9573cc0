// pg_edges.hip -- aggregation operators (edge weights, direct terms) and the
// per-path pass (successors, predecessors, path-traced initial estimate).
//
// Paper Sec. "Path Graph Operators": each neighbour of a receiver is a
// sampling technique; its continuation sample is combined with the balance
// heuristic over all techniques of the receiver's neighbourhood (eqs.
// indirect-weight, ag-indirect), and the direct-light records form 2K samples
// from K+1 strategies (eq. ag-direct).  The pdfs of the techniques are HG
// with parameter g_s about each neighbour's arriving direction; the receiver
// evaluates its own phase function (HG with g about its arriving direction).
#include "pg_internal.h"

namespace pg {

__device__ inline f3 rec_f3(const float* p) { return f3{p[0], p[1], p[2]}; }

// One group of KP lanes per receiver, lane j = j-th neighbour.  The
// neighbours' arriving directions (the techniques) are staged in LDS; every
// lane sums the K technique pdfs at its own two samples (continuation and
// environment) to get the marginals, then forms its three weights; the
// direct term is a group reduction.
template <int KP>
__global__ __launch_bounds__(kBlock) void k_edges(int64_t N, Consts c, const int32_t* __restrict__ col,
                                                  const VRec* __restrict__ rec, EdgeOut o, int32_t* flag) {
    constexpr int GR = kBlock / KP;
    __shared__ f3 tsh[GR][KP];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % KP, grp = threadIdx.x / KP;
    const int64_t i = tile * GR + grp;
    const int K = c.K;
    const bool row_ok = i < N;
    bool act = row_ok && lane < K;

    f3 t{0.f, 0.f, 0.f}, w{0.f, 0.f, 0.f}, we{0.f, 0.f, 0.f}, ls{0.f, 0.f, 0.f}, le{0.f, 0.f, 0.f},
        lp{0.f, 0.f, 0.f};
    float alpha = 0.0f;
    f3 dpl{0.f, 0.f, 0.f}, lpl{0.f, 0.f, 0.f};   // point light sample of the neighbour
    const int64_t e = o.ell ? eidx(i, lane, K) : i * K + lane;
    if (act) {
        int64_t j = col[e];
        if (j < 0 || j >= N || (lane == 0 && j != i)) {
            set_flag(flag, kFlagIndex);
            act = false;
        } else {
            const float4* r4 = reinterpret_cast<const float4*>(rec + j);
            float4 a0 = r4[0], a1 = r4[1], a2 = r4[2], a3 = r4[3], a4 = r4[4];
            t = f3{a0.x, a0.y, a0.z};
            w = f3{a0.w, a1.x, a1.y};
            we = f3{a1.z, a1.w, a2.x};
            ls = f3{a2.y, a2.z, a2.w};
            le = f3{a3.x, a3.y, a3.z};
            lp = f3{a3.w, a4.x, a4.y};
            alpha = a4.z;
            if (o.dir_pl) {
                const int64_t cj = o.canon_row ? (int64_t)o.canon_row[j] : j;
                dpl = ld3(o.dir_pl, cj);
                lpl = ld3(o.l_pl, cj);
            }
        }
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
    const float wi = rho / mplus;
    const float wp = rho / (mplus + Kpe);
    const float wev = rho_e / (menv + Kpe);

    float cx = act ? wev * le.x + wp * lp.x : 0.0f;
    float cy = act ? wev * le.y + wp * lp.y : 0.0f;
    float cz = act ? wev * le.z + wp * lp.z : 0.0f;
    float sx = act ? ls.x : 0.0f, sy = act ? ls.y : 0.0f, sz = act ? ls.z : 0.0f;
    cx = group_sum<KP>(cx);
    cy = group_sum<KP>(cy);
    cz = group_sum<KP>(cz);
    sx = group_sum<KP>(sx);
    sy = group_sum<KP>(sy);
    sz = group_sum<KP>(sz);
    // point light: a delta light per neighbour sample, weight 1/K
    const float rho_pl = (act && o.dir_pl) ? c.rho(one_minus_cos(ti, dpl)) : 0.0f;
    float qx = rho_pl * lpl.x, qy = rho_pl * lpl.y, qz = rho_pl * lpl.z;
    if (o.dir_pl) {
        qx = group_sum<KP>(qx);
        qy = group_sum<KP>(qy);
        qz = group_sum<KP>(qz);
    }

    if (o.ell && row_ok && lane == 0) {   // padding slots of the last quad: weight 0
        for (int l = K; l < ell_k4(K); ++l) {
            o.w[eidx(i, l, K)] = 0.0f;
            if (o.gw) o.gw[eidx(i, l, K)] = 0.0f;
        }
    }
    if (act) {
        o.w[e] = wi;
        if (o.gw) o.gw[e] = wi * hg_dlog(c.g, u_w);
        if (o.canon_row || o.w_ind || o.w_ph || o.w_env) {
            const int64_t ce = (o.canon_row ? (int64_t)o.canon_row[i] : i) * K + lane;
            if (o.w_ind) o.w_ind[ce] = wi;
            if (o.w_ph) o.w_ph[ce] = wp;
            if (o.w_env) o.w_env[ce] = wev;
        }
    }
    if (row_ok && lane == 0) {
        // aggregated direct: sun (delta light, weight 1/K per neighbour) + MIS'd records
        const float rho_sun = c.rho(one_minus_cos(ti, c.sun));
        const float invK = 1.0f / (float)K;
        f3 dagg{fmaf(rho_sun * invK, sx, cx), fmaf(rho_sun * invK, sy, cy), fmaf(rho_sun * invK, sz, cz)};
        if (o.dir_pl) dagg = f3{fmaf(invK, qx, dagg.x), fmaf(invK, qy, dagg.y), fmaf(invK, qz, dagg.z)};
        // constant of the row: the vertex's own volume emission (not scattered) + alpha d_agg
        f3 em{0.f, 0.f, 0.f};
        if (o.emit) em = ld3(o.emit, o.canon_row ? (int64_t)o.canon_row[i] : i);
        const f3 b{fmaf(alpha, dagg.x, em.x), fmaf(alpha, dagg.y, em.y), fmaf(alpha, dagg.z, em.z)};
        // own (path-traced) direct: one sun sample, environment and phase samples by the balance heuristic
        const float p_w = c.pdf(u_w), p_e = c.pdf(u_e);
        const float f_env = rho_e / (p_e + c.env_pdf), f_out = rho / (p_w + c.env_pdf);
        f3 dpt{rho_sun * ls.x + f_env * le.x + f_out * lp.x, rho_sun * ls.y + f_env * le.y + f_out * lp.y,
               rho_sun * ls.z + f_env * le.z + f_out * lp.z};
        if (o.dir_pl)   // lane 0 holds the receiver's own sample
            dpt = f3{fmaf(rho_pl, lpl.x, dpt.x), fmaf(rho_pl, lpl.y, dpt.y), fmaf(rho_pl, lpl.z, dpt.z)};
        st3(o.b, i, b);
        st3(o.dpt, i, dpt);
        o.r[i] = rho / p_w;
        o.alpha[i] = alpha;
        if (o.b_canon || o.dpt_canon) {
            const int64_t ci = o.canon_row ? (int64_t)o.canon_row[i] : i;
            if (o.b_canon) st3(o.b_canon, ci, b);
            if (o.dpt_canon) st3(o.dpt_canon, ci, dpt);
        }
    }
}

hipError_t launch_edges(int64_t N, const Consts& c, const int32_t* col, const VRec* rec, const EdgeOut& o,
                        int32_t* flag, hipStream_t s) {
    if (N == 0) return hipSuccess;
    dispatch_kp(c.K, [&](auto kp) {
        constexpr int KP = decltype(kp)::value;
        hipLaunchKernelGGL(k_edges<KP>, dim3((unsigned)div_up(N, kBlock / KP)), dim3(kBlock), 0, s, N, c, col,
                           rec, o, flag);
    });
    return hipGetLastError();
}

// One wave per path.  Writes, in local ids, succ(v) / pred(v) (-1 at the
// ends) and the initial radiance arriving from the successor u along the
// continuation: 0 at the last vertex, else e_u + albedo_u (d_pt_u + r_u L(u))
// -- the path tracer's own estimate (init PT) -- or e_u alone (init zero: the
// indirect part starts at 0), e_u being the volume emission collected at u
// (emit, path order, nullable: 0).  The recurrence L(v) = F_u(L(u)), F_u an
// affine map, is taken 64 vertices at a time from the path's end: lane c
// holds vertex hi - c, a wave-level inclusive scan composes the lanes' maps
// (F(L) = A + B L; F2 o F1 = (A2 + B2 A1, B2 B1)), and each lane applies
// the composition of the lanes above it to the value arriving at the chunk.
// succ, pred and x0 must be pre-filled with -1, -1, 0.
__global__ __launch_bounds__(kBlock) void k_paths(int64_t P, int64_t N, const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ inv, const float* __restrict__ alpha,
                                                  const float* __restrict__ dpt, const float* __restrict__ r,
                                                  const float* __restrict__ emit, int init,
                                                  int32_t* __restrict__ succ, int32_t* __restrict__ pred,
                                                  float* __restrict__ x0, int32_t* flag) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;   // uniform over the wave
    if (p == 0 && lane == 0 && (off[0] != 0 || off[P] != N)) set_flag(flag, kFlagOffsets);
    if (p >= P) return;
    const int64_t a = off[p], e = off[p + 1];
    if (a < 0 || e < a || e > N) {
        if (lane == 0) set_flag(flag, kFlagOffsets);
        return;
    }
    const bool pt = init == PG_INIT_PT && x0;
    const bool ez = !pt && emit && x0;   // init zero with emission
    auto sid = [&](int64_t u) { return inv ? inv[u] : (int32_t)u; };
    f3 carry{0.f, 0.f, 0.f};   // the value arriving at the chunk's highest vertex
    for (int64_t hi = e - 1; hi >= a; hi -= kWave) {
        const int64_t v = hi - lane;
        const bool valid = v >= a;
        const int32_t s = valid ? sid(v) : -1;
        if (valid) {
            if (succ) succ[s] = v + 1 < e ? sid(v + 1) : -1;
            if (pred) pred[s] = v > a ? sid(v - 1) : -1;
        }
        if (!pt && !ez) continue;
        // this vertex's map: the value arriving at its predecessor from the
        // value arriving at it (identity on the lanes past the path's start)
        float B = 1.0f;
        f3 A{0.f, 0.f, 0.f};
        if (valid) {
            const f3 em = emit ? ld3(emit, v) : f3{0.f, 0.f, 0.f};
            if (pt) {
                const float al = alpha[s];
                const f3 d = ld3(dpt, s);
                B = al * r[s];
                A = f3{fmaf(al, d.x, em.x), fmaf(al, d.y, em.y), fmaf(al, d.z, em.z)};
            } else {
                B = 0.0f;
                A = em;
            }
        }
        // inclusive scan: lane c composes the maps of lanes 0..c (lane c's
        // applied last)
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const float Bo = __shfl_up(B, o, kWave);
            const float Ax = __shfl_up(A.x, o, kWave), Ay = __shfl_up(A.y, o, kWave), Az = __shfl_up(A.z, o, kWave);
            if (lane >= o) {
                A = f3{fmaf(B, Ax, A.x), fmaf(B, Ay, A.y), fmaf(B, Az, A.z)};
                B *= Bo;
            }
        }
        // exclusive: the lanes above this one, applied to the carry
        // every lane takes part in the shuffles (a lane inactive in one
        // gives no data to its neighbour), then lane 0 takes the identity
        const float Bsh = __shfl_up(B, 1, kWave);
        const float Be = lane > 0 ? Bsh : 1.0f;
        const float Aex = __shfl_up(A.x, 1, kWave), Aey = __shfl_up(A.y, 1, kWave), Aez = __shfl_up(A.z, 1, kWave);
        const f3 Ae = lane > 0 ? f3{Aex, Aey, Aez} : f3{0.f, 0.f, 0.f};
        if (valid) st3(x0, s, f3{fmaf(Be, carry.x, Ae.x), fmaf(Be, carry.y, Ae.y), fmaf(Be, carry.z, Ae.z)});
        // the value arriving at the next chunk's highest vertex (the whole
        // chunk's composition, held by lane 63)
        const float Bl = __shfl(B, kWave - 1, kWave);
        const f3 Al{__shfl(A.x, kWave - 1, kWave), __shfl(A.y, kWave - 1, kWave), __shfl(A.z, kWave - 1, kWave)};
        carry = f3{fmaf(Bl, carry.x, Al.x), fmaf(Bl, carry.y, Al.y), fmaf(Bl, carry.z, Al.z)};
    }
}

hipError_t launch_paths(int64_t P, int64_t N, const int64_t* off, const int32_t* inv, const float* alpha,
                        const float* dpt, const float* r, const float* emit, int init, int32_t* succ, int32_t* pred,
                        float* x0, int32_t* flag, hipStream_t s) {
    const int64_t n = P > 0 ? P : 1;
    hipLaunchKernelGGL(k_paths, dim3((unsigned)div_up(n * kWave, kBlock)), dim3(kBlock), 0, s, P, N, off, inv, alpha,
                       dpt, r, emit, init, succ, pred, x0, flag);
    return hipGetLastError();
}

}  // namespace pg
