// pg_clusters.hip -- the paper's own neighbour relation: disjoint clusters
// around random centres (Sec. "Path Graph Framework"; Sec. "Rendering
// System", path graph solver), and the aggregation over them.
//
// Clusters.  Vertex i is a centre when its caller-drawn uniform 32-bit key is
// below floor(2^32 / K) (about N/K centres); the vertex with the smallest
// (key, path id) always is one.  Every vertex joins the nearest centre by
// (squared distance of the 20-bit quantised positions, centre path id),
// found by a ring search over a uniform grid of the centres alone.  A
// cluster with more than 2K members takes its ceil(s/K) members of smallest
// (key, path id) as new centres and its members join the nearest of those;
// this repeats up to kClusterRounds rounds for the clusters still large.
//
// Layout.  The render then runs in "cluster order": clusters one after the
// other (ordered by their centre's place in the spatially sorted order), the
// members of a cluster by ascending path id.  A row's neighbours are exactly
// its cluster's members, a contiguous range [a, e).
//
// Aggregation.  All receivers of a cluster combine the same techniques, so
// the marginal density of a sample is one number per sample (first pass,
// O(C) per vertex), and the weight w+_ij = rho_i(w_j) / M+(w_j) is
// recomputed in every iteration from the receiver's arriving direction and
// the member's (w_j, 1/M+_j) instead of being stored: per iteration a row
// reads 16 + 12 + 12 bytes of its own and its cluster's members' 16 + 12
// bytes from L1/L2 (the members are contiguous and shared by the wave's
// rows), against 8 bytes per edge plus a gather for the stored sliced ELL.
#include <algorithm>
#include <utility>

#include "pg_api_common.h"

namespace pg {

namespace {

__device__ inline int64_t qdist2(uint64_t a, uint64_t b) {
    int32_t ax, ay, az, bx, by, bz;
    qunpack(a, ax, ay, az);
    qunpack(b, bx, by, bz);
    const int64_t dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

__device__ inline bool near_less(int64_t d1, int32_t p1, int64_t d2, int32_t p2) {
    return d1 < d2 || (d1 == d2 && p1 < p2);
}

// ------------------------------------------------------------- centres ---

__device__ inline unsigned long long wave_min(unsigned long long m) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(m, o, kWave);
        m = t < m ? t : m;
    }
    return m;
}

// min over all vertices of (key << 32 | path id): one partial per block ...
__global__ __launch_bounds__(kBlock) void k_key_min(int64_t N, const uint32_t* __restrict__ key,
                                                    unsigned long long* __restrict__ part) {
    __shared__ unsigned long long sm[kBlock / kWave];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long m = v < N ? ((unsigned long long)key[v] << 32) | (unsigned long long)v : ~0ull;
    m = wave_min(m);
    if (__lane_id() == 0) sm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) m = sm[w] < m ? sm[w] : m;
        part[blockIdx.x] = m;
    }
}

// ... then one block over the partials
__global__ __launch_bounds__(1024) void k_key_min_final(int64_t n, const unsigned long long* __restrict__ part,
                                                        unsigned long long* __restrict__ kmin) {
    __shared__ unsigned long long sm[1024 / kWave];
    unsigned long long m = ~0ull;
    for (int64_t t = threadIdx.x; t < n; t += 1024) m = part[t] < m ? part[t] : m;
    m = wave_min(m);
    if (__lane_id() == 0) sm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / kWave; ++w) m = sm[w] < m ? sm[w] : m;
        *kmin = m;
    }
}

// Is sorted vertex s a centre?
__device__ inline bool is_centre(int32_t pid, const uint32_t* __restrict__ key, unsigned long long thr,
                                 const unsigned long long* __restrict__ kmin) {
    return (unsigned long long)key[pid] < thr || (uint32_t)(*kmin & 0xffffffffull) == (uint32_t)pid;
}

// Adds one to counter[k] for every active lane and returns the lane's slot:
// the counter's old value plus the lane's rank among the lanes with the
// same k.  One atomic per distinct k in the wave (ballots group the lanes).
__device__ inline uint32_t wave_count(uint32_t* counter, int32_t k) {
    uint64_t todo = __ballot(1);
    const int lane = (int)__lane_id();
    uint32_t mine = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t kl = __shfl(k, leader, kWave);
        const uint64_t m = __ballot(k == kl) & todo;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&counter[kl], (uint32_t)__popcll(m));
        base = (uint32_t)__shfl((int)base, leader, kWave);
        if ((m >> lane) & 1ull) mine = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        todo &= ~m;
    }
    return mine;
}

__device__ inline uint32_t cg_cell(uint64_t q, int b) {
    int32_t x, y, z;
    qunpack(q, x, y, z);
    const int sh = kQBits - b;
    return ((uint32_t)(z >> sh) << (2 * b)) | ((uint32_t)(y >> sh) << b) | (uint32_t)(x >> sh);
}

__global__ __launch_bounds__(kBlock) void k_cg_count(int64_t N, const int32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ key, unsigned long long thr,
                                                     const unsigned long long* __restrict__ kmin,
                                                     const uint64_t* __restrict__ qs, int b,
                                                     uint32_t* __restrict__ gcount, uint32_t* __restrict__ gcell,
                                                     uint32_t* __restrict__ grank) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N || !is_centre(perm[s], key, thr, kmin)) return;
    const uint32_t cell = cg_cell(qs[s], b);
    gcell[s] = cell;
    grank[s] = atomicAdd(&gcount[cell], 1u);
}

__global__ __launch_bounds__(kBlock) void k_cg_scatter(int64_t N, const int32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ key, unsigned long long thr,
                                                       const unsigned long long* __restrict__ kmin,
                                                       const uint64_t* __restrict__ qs,
                                                       const uint32_t* __restrict__ gcell,
                                                       const uint32_t* __restrict__ grank,
                                                       const uint32_t* __restrict__ gstart, uint64_t* __restrict__ gq,
                                                       int32_t* __restrict__ gs, int32_t* __restrict__ gpid) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int32_t pid = perm[s];
    if (!is_centre(pid, key, thr, kmin)) return;
    const uint32_t pos = gstart[gcell[s]] + grank[s];
    gq[pos] = qs[s];
    gs[pos] = (int32_t)s;
    gpid[pos] = pid;
}

// Nearest centre of every vertex: rings of cells at Chebyshev distance r
// around the vertex's cell, r = 0, 1, ....  A cell whose box is farther than
// the best distance so far is skipped (one at exactly that distance is read:
// a tie may win on its path id).  After ring r every unvisited centre is at
// least `gap` quantisation steps away on some axis, so the search ends once
// the best squared distance is below gap^2.
__global__ __launch_bounds__(kBlock) void k_nearest_centre(int64_t N, const uint64_t* __restrict__ qs, int b,
                                                           const uint32_t* __restrict__ gstart,
                                                           const uint64_t* __restrict__ gq,
                                                           const int32_t* __restrict__ gs,
                                                           const int32_t* __restrict__ gpid,
                                                           int32_t* __restrict__ cid, int32_t* flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const uint64_t q = qs[s];
    int32_t qx, qy, qz;
    qunpack(q, qx, qy, qz);
    const int sh = kQBits - b;
    const int side = 1 << b;
    const int cx = qx >> sh, cy = qy >> sh, cz = qz >> sh;
    int64_t bd = INT64_MAX;
    int32_t bp = INT32_MAX, bs = -1;
    const int64_t cw = (int64_t)1 << sh;   // cell width in quantisation steps
    for (int r = 0; r < side; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= side) continue;
            const int64_t gz = dz < 0 ? (int64_t)qz - ((int64_t)(z + 1) * cw - 1) : (dz > 0 ? (int64_t)z * cw - qz : 0);
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= side) continue;
                const int64_t gy = dy < 0 ? (int64_t)qy - ((int64_t)(y + 1) * cw - 1) : (dy > 0 ? (int64_t)y * cw - qy : 0);
                const bool face = dz == -r || dz == r || dy == -r || dy == r;
                const int step = face ? 1 : 2 * r;
                for (int dx = -r; dx <= r; dx += step) {
                    const int x = cx + dx;
                    if (x < 0 || x >= side) continue;
                    const int64_t gx = dx < 0 ? (int64_t)qx - ((int64_t)(x + 1) * cw - 1) : (dx > 0 ? (int64_t)x * cw - qx : 0);
                    if (gx * gx + gy * gy + gz * gz > bd) continue;   // the whole cell is farther
                    const uint32_t cell = ((uint32_t)z << (2 * b)) | ((uint32_t)y << b) | (uint32_t)x;
                    const uint32_t e1 = gstart[cell + 1];
                    for (uint32_t e = gstart[cell]; e < e1; ++e) {
                        const int64_t d2 = qdist2(q, gq[e]);
                        const int32_t p = gpid[e];
                        if (near_less(d2, p, bd, bp)) {
                            bd = d2;
                            bp = p;
                            bs = gs[e];
                        }
                    }
                }
            }
        }
        // smallest per-axis distance from q to a cell outside the searched cube
        int64_t gap = INT64_MAX;
        const int c3[3] = {cx, cy, cz};
        const int64_t q3[3] = {qx, qy, qz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c3[a] - r > 0) gap = min(gap, q3[a] - (int64_t)(c3[a] - r) * cw + 1);
            if (c3[a] + r < side - 1) gap = min(gap, (int64_t)(c3[a] + r + 1) * cw - q3[a]);
        }
        if (gap == INT64_MAX) break;                // the whole grid was searched
        if (bs >= 0 && bd < gap * gap) break;       // provably final
    }
    if (bs < 0) set_flag(flag, kFlagCluster);
    cid[s] = bs < 0 ? (int32_t)s : bs;
}

// ------------------------------------------------------------ grouping ---

__global__ __launch_bounds__(kBlock) void k_ccount(int64_t N, const int32_t* __restrict__ cid,
                                                   uint32_t* __restrict__ ccount) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < N) (void)wave_count(ccount, cid[s]);
}

// Groups the vertices by centre.  Besides the sorted id, each slot keeps
// the member's (key << 32 | path id) and packed position, so that the loops
// over a group read contiguous memory.
__global__ __launch_bounds__(kBlock) void k_cgroup(int64_t N, const int32_t* __restrict__ cid,
                                                   const uint32_t* __restrict__ cstart, uint32_t* __restrict__ cfill,
                                                   const int32_t* __restrict__ perm, const uint32_t* __restrict__ key,
                                                   const uint64_t* __restrict__ qs, int32_t* __restrict__ members,
                                                   uint32_t* __restrict__ mslot, unsigned long long* __restrict__ mkey,
                                                   uint64_t* __restrict__ mq) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int32_t c = cid[s];
    const uint32_t slot = cstart[c] + wave_count(cfill, c);
    const int32_t pid = perm[s];
    members[slot] = (int32_t)s;
    mslot[s] = slot;
    mkey[slot] = ((unsigned long long)key[pid] << 32) | (uint32_t)pid;
    mq[slot] = qs[s];
}

// A cluster above kClusterMax members is reported (kFlagCluster) and its
// rows are left empty, so that no loop runs over it.
__device__ inline uint2 bounded(uint2 rg) {
    if (rg.y - rg.x > (uint32_t)kClusterMax) rg.y = rg.x;
    return rg;
}

// ----------------------------------------------------------- splitting ---

// Members of a large cluster: the ceil(s/K) of smallest (key, path id)
// become centres (newc, by group slot).  O(s) per member.  The cluster's
// centre is appended to the round's list of split clusters.
__global__ __launch_bounds__(kBlock) void k_split_mark(int64_t N, int K, const int32_t* __restrict__ cid,
                                                       const uint32_t* __restrict__ ccount,
                                                       const uint32_t* __restrict__ cstart,
                                                       const uint32_t* __restrict__ mslot,
                                                       const unsigned long long* __restrict__ mkey,
                                                       uint8_t* __restrict__ newc, const int32_t* __restrict__ live,
                                                       int32_t* __restrict__ split, uint32_t* __restrict__ nsplit,
                                                       int32_t* __restrict__ splitlist, int32_t* flag) {
    if (live && *live == 0) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int32_t c = cid[s];
    const uint32_t sz = ccount[c];
    if (sz <= 2u * (uint32_t)K) return;
    if (sz > (uint32_t)kClusterMax) {
        set_flag(flag, kFlagCluster);
        return;
    }
    const uint32_t me = mslot[s];
    const unsigned long long mine = mkey[me];
    const uint32_t a = cstart[c];
    uint32_t rank = 0;
    for (uint32_t e = a; e < a + sz; ++e) rank += mkey[e] < mine;
    newc[me] = rank < (sz + (uint32_t)K - 1u) / (uint32_t)K;
    if (__lane_id() == (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1)) *split = 1;
    const bool first = me == a;   // one member per split cluster lists it
    const uint32_t at = wave_append(nsplit, first);
    if (first) splitlist[at] = c;
}

// Members of a large cluster join the nearest of its new centres.
__global__ __launch_bounds__(kBlock) void k_split_assign(int64_t N, int K, const uint64_t* __restrict__ qs,
                                                         int32_t* __restrict__ cid, const uint32_t* __restrict__ ccount,
                                                         const uint32_t* __restrict__ cstart,
                                                         const int32_t* __restrict__ members,
                                                         const unsigned long long* __restrict__ mkey,
                                                         const uint64_t* __restrict__ mq,
                                                         const uint8_t* __restrict__ newc,
                                                         const int32_t* __restrict__ live) {
    if (live && *live == 0) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int32_t c = cid[s];
    const uint32_t sz = ccount[c];
    if (sz <= 2u * (uint32_t)K || sz > (uint32_t)kClusterMax) return;
    const uint64_t q = qs[s];
    const uint32_t a = cstart[c];
    int64_t bd = INT64_MAX;
    int32_t bp = INT32_MAX;
    uint32_t be = a;
    for (uint32_t e = a; e < a + sz; ++e) {
        if (!newc[e]) continue;
        const int64_t d2 = qdist2(q, mq[e]);
        const int32_t p = (int32_t)(mkey[e] & 0xffffffffull);
        if (near_less(d2, p, bd, bp)) {
            bd = d2;
            bp = p;
            be = e;
        }
    }
    cid[s] = members[be];
}

// Exclusive prefix sum over the block's threads; total = the block's sum.
__device__ inline uint32_t block_scan_excl(uint32_t v, uint32_t& total, uint32_t* wsum) {
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x / kWave);
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        const uint32_t t = wsum[i];
        off += i < w ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// After a split round, each split cluster is regrouped inside its own slot
// range [a, a + size): its members joined new centres drawn from the same
// cluster, so the new clusters partition that range and every other
// cluster's grouping stays valid.  One block per split cluster (grid-stride
// over the round's list).  The range is staged (same slots) and written back
// grouped by new centre, in the slot order of the new centres; within a new
// cluster the order is that of the block's atomics, as in the global
// grouping (every later step ranks the members by key or path id).
__global__ __launch_bounds__(kBlock) void k_regroup(const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ nlist,
                                                    const int32_t* __restrict__ cid, uint32_t* __restrict__ ccount,
                                                    uint32_t* __restrict__ cstart, int32_t* __restrict__ members,
                                                    uint32_t* __restrict__ mslot,
                                                    unsigned long long* __restrict__ mkey, uint64_t* __restrict__ mq,
                                                    const uint8_t* __restrict__ newc, int32_t* __restrict__ stage_m,
                                                    unsigned long long* __restrict__ stage_k,
                                                    uint64_t* __restrict__ stage_q) {
    __shared__ uint32_t s_cnt[kClusterMax];     // members per new centre, then fill counters
    __shared__ uint32_t s_start[kClusterMax];   // first local slot of each new centre
    __shared__ int32_t s_cent[kClusterMax];     // sorted id of each new centre
    __shared__ uint16_t s_pre[kClusterMax];     // new centres in the local slots before t
    __shared__ uint16_t s_idx[kClusterMax];     // each member's new-centre index
    __shared__ uint32_t s_wsum[kBlock / kWave];
    const uint32_t n = *nlist;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const int32_t c = list[it];
        const uint32_t a = cstart[c], sz = ccount[c];   // 2K < sz <= kClusterMax (split clusters only)
        // the new centres in slot order, and the range staged
        uint32_t nc = 0;
        for (uint32_t base = 0; base < sz; base += kBlock) {
            const uint32_t t = base + threadIdx.x;
            const bool in = t < sz;
            const uint32_t f = (in && newc[a + t]) ? 1u : 0u;
            uint32_t tot;
            const uint32_t pre = nc + block_scan_excl(f, tot, s_wsum);
            if (in) {
                const int32_t m = members[a + t];
                s_pre[t] = (uint16_t)pre;
                if (f) s_cent[pre] = m;
                stage_m[a + t] = m;
                stage_k[a + t] = mkey[a + t];
                stage_q[a + t] = mq[a + t];
            }
            nc += tot;
        }
        for (uint32_t j = threadIdx.x; j < nc; j += kBlock) s_cnt[j] = 0;
        __syncthreads();
        // members per new centre (a new centre's slot is still its old one)
        for (uint32_t t = threadIdx.x; t < sz; t += kBlock) {
            const uint32_t j = s_pre[mslot[cid[stage_m[a + t]]] - a];
            s_idx[t] = (uint16_t)j;
            atomicAdd(&s_cnt[j], 1u);
        }
        __syncthreads();
        uint32_t run = 0;
        for (uint32_t base = 0; base < nc; base += kBlock) {
            const uint32_t j = base + threadIdx.x;
            uint32_t tot;
            const uint32_t pre = run + block_scan_excl(j < nc ? s_cnt[j] : 0u, tot, s_wsum);
            if (j < nc) s_start[j] = pre;
            run += tot;
        }
        for (uint32_t j = threadIdx.x; j < nc; j += kBlock) {
            ccount[s_cent[j]] = s_cnt[j];
            cstart[s_cent[j]] = a + s_start[j];
            s_cnt[j] = 0;
        }
        __syncthreads();
        // write back grouped by new centre
        for (uint32_t t = threadIdx.x; t < sz; t += kBlock) {
            const uint32_t j = s_idx[t];
            const uint32_t e = a + s_start[j] + atomicAdd(&s_cnt[j], 1u);
            const int32_t m = stage_m[a + t];
            members[e] = m;
            mkey[e] = stage_k[a + t];
            mq[e] = stage_q[a + t];
            mslot[m] = e;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- the order ---

// Cluster order: position = cluster start + rank of the path id among the
// members.  Writes cperm (position -> sorted id), cinv (path id -> position)
// and each position's member range.
__global__ __launch_bounds__(kBlock) void k_corder(int64_t N, const int32_t* __restrict__ cid,
                                                   const uint32_t* __restrict__ ccount,
                                                   const uint32_t* __restrict__ cstart,
                                                   const uint32_t* __restrict__ mslot,
                                                   const unsigned long long* __restrict__ mkey,
                                                   const int32_t* __restrict__ perm, int32_t* __restrict__ cperm,
                                                   int32_t* __restrict__ cinv, uint2* __restrict__ crange,
                                                   int32_t* flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t sz = 0;
    if (s < N) {
        const int32_t c = cid[s];
        sz = ccount[c];
        const uint32_t a = cstart[c];
        const int32_t pid = perm[s];
        uint32_t rank = 0;
        if (sz > (uint32_t)kClusterMax) {
            set_flag(flag, kFlagCluster);   // not ranked: the result is reported invalid
            rank = mslot[s] - a;
        } else {
            for (uint32_t e = a; e < a + sz; ++e) rank += (int32_t)(mkey[e] & 0xffffffffull) < pid;
        }
        const uint32_t pos = a + rank;
        cperm[pos] = (int32_t)s;
        cinv[pid] = (int32_t)pos;
        crange[pos] = make_uint2(a, a + sz);
    }
}

// Records in cluster order, plus (t, alpha) packed for the iteration.
__global__ __launch_bounds__(kBlock) void k_crec(int64_t N, const int32_t* __restrict__ cperm,
                                                 const VRec* __restrict__ rec, VRec* __restrict__ crec,
                                                 float4* __restrict__ tq, float* __restrict__ alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4* src = reinterpret_cast<const float4*>(rec + cperm[i]);
    float4* dst = reinterpret_cast<float4*>(crec + i);
    float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3], a4 = src[4];
    dst[0] = a0;
    dst[1] = a1;
    dst[2] = a2;
    dst[3] = a3;
    dst[4] = a4;
    tq[i] = make_float4(a0.x, a0.y, a0.z, a4.z);
    alpha[i] = a4.z;
}

// --------------------------------------------------------- the weights ---

// First pass: the marginals of every vertex's own samples over its cluster,
//   M+(w_i) = sum_l p_l(w_i),  Me(we_i) = sum_l p_l(we_i) + C p_e,
// stored as wq = (w_i, c_g / M+) with c_g = (1 - g^2) / (4 pi) the HG
// constant, mp = M+ + C p_e, me = Me.
__global__ __launch_bounds__(kBlock) void k_cmarg(int64_t N, Consts c, const uint2* __restrict__ crange,
                                                  const VRec* __restrict__ crec, const float4* __restrict__ tq,
                                                  float4* __restrict__ wq, float* __restrict__ mp,
                                                  float* __restrict__ me) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint2 rg = bounded(crange[i]);
    const VRec& ri = crec[i];
    const f3 w{ri.w[0], ri.w[1], ri.w[2]}, we{ri.we[0], ri.we[1], ri.we[2]};
    float mplus = 0.0f, menv = 0.0f;
    for (uint32_t l = rg.x; l < rg.y; ++l) {
        const float4 t4 = tq[l];
        const f3 tl{t4.x, t4.y, t4.z};
        mplus += c.pdf(one_minus_cos(tl, w));
        menv += c.pdf(one_minus_cos(tl, we));
    }
    const float Cpe = (float)(rg.y - rg.x) * c.env_pdf;
    wq[i] = make_float4(w.x, w.y, w.z, c.rho.c / mplus);
    mp[i] = mplus + Cpe;
    me[i] = menv + Cpe;
}

// Second pass, per receiver i over its cluster's samples j:
//   d_agg_i = rho_i(sun)/C sum_j Ls_j + sum_j rho_i(we_j) Le_j / Me_j + rho_i(w_j) Lp_j / (M+_j + C p_e)
//   b_i = e_i + alpha_i d_agg_i,  and the own (path-traced) direct term and ratio.
__global__ __launch_bounds__(kBlock) void k_cedges(int64_t N, Consts c, const uint2* __restrict__ crange,
                                                   const VRec* __restrict__ crec, const float4* __restrict__ tq,
                                                   const float* __restrict__ mp, const float* __restrict__ me,
                                                   const float* __restrict__ emit, const int32_t* __restrict__ cperm,
                                                   const int32_t* __restrict__ perm, const float* __restrict__ dir_pl,
                                                   const float* __restrict__ l_pl, float* __restrict__ b,
                                                   float* __restrict__ dpt, float* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint2 rg = bounded(crange[i]);
    const float4 t4 = tq[i];
    const f3 ti{t4.x, t4.y, t4.z};
    float cx = 0.f, cy = 0.f, cz = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, qx = 0.f, qy = 0.f, qz = 0.f;
    for (uint32_t j = rg.x; j < rg.y; ++j) {
        const VRec& rj = crec[j];
        const f3 wj{rj.w[0], rj.w[1], rj.w[2]}, wej{rj.we[0], rj.we[1], rj.we[2]};
        const float fp = c.rho(one_minus_cos(ti, wj)) / mp[j];
        const float fe = c.rho(one_minus_cos(ti, wej)) / me[j];
        cx += fe * rj.le[0] + fp * rj.lp[0];
        cy += fe * rj.le[1] + fp * rj.lp[1];
        cz += fe * rj.le[2] + fp * rj.lp[2];
        sx += rj.ls[0];
        sy += rj.ls[1];
        sz += rj.ls[2];
        if (dir_pl) {   // point light: a delta light per member sample, weight 1/C
            const int64_t pj = perm[cperm[j]];
            const float rp = c.rho(one_minus_cos(ti, ld3(dir_pl, pj)));
            const f3 lq = ld3(l_pl, pj);
            qx = fmaf(rp, lq.x, qx);
            qy = fmaf(rp, lq.y, qy);
            qz = fmaf(rp, lq.z, qz);
        }
    }
    const float rho_sun = c.rho(one_minus_cos(ti, c.sun));
    const float invC = 1.0f / (float)(rg.y - rg.x);
    f3 dagg{fmaf(rho_sun * invC, sx, cx), fmaf(rho_sun * invC, sy, cy), fmaf(rho_sun * invC, sz, cz)};
    if (dir_pl) dagg = f3{fmaf(invC, qx, dagg.x), fmaf(invC, qy, dagg.y), fmaf(invC, qz, dagg.z)};
    f3 em{0.f, 0.f, 0.f};
    if (emit) em = ld3(emit, perm[cperm[i]]);
    const float al = t4.w;
    st3(b, i, f3{fmaf(al, dagg.x, em.x), fmaf(al, dagg.y, em.y), fmaf(al, dagg.z, em.z)});
    const VRec& ri = crec[i];
    const f3 w{ri.w[0], ri.w[1], ri.w[2]}, we{ri.we[0], ri.we[1], ri.we[2]};
    const float u_w = one_minus_cos(ti, w), u_e = one_minus_cos(ti, we);
    const float rho = c.rho(u_w), rho_e = c.rho(u_e);
    const float p_w = c.pdf(u_w), p_e = c.pdf(u_e);
    const float f_env = rho_e / (p_e + c.env_pdf), f_out = rho / (p_w + c.env_pdf);
    f3 dp{rho_sun * ri.ls[0] + f_env * ri.le[0] + f_out * ri.lp[0],
          rho_sun * ri.ls[1] + f_env * ri.le[1] + f_out * ri.lp[1],
          rho_sun * ri.ls[2] + f_env * ri.le[2] + f_out * ri.lp[2]};
    if (dir_pl) {
        const int64_t pi = perm[cperm[i]];
        const float rp = c.rho(one_minus_cos(ti, ld3(dir_pl, pi)));
        const f3 lq = ld3(l_pl, pi);
        dp = f3{fmaf(rp, lq.x, dp.x), fmaf(rp, lq.y, dp.y), fmaf(rp, lq.z, dp.z)};
    }
    st3(dpt, i, dp);
    r[i] = rho / p_w;
}

// ------------------------------------------------------- the iteration ---

// HG_g(t, w) / c_g = ((1-g)^2 + g |t - w|^2)^(-3/2), the receiver's phase
// without its constant (which the member's wq.w carries).
__device__ __forceinline__ float hg_shape(const HG& rho, f3 t, float wx, float wy, float wz) {
    const float dx = t.x - wx, dy = t.y - wy, dz = t.z - wz;
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float r = __frsqrt_rn(fmaf(0.5f * rho.two_g, d2, rho.a));
    return r * r * r;
}

// The shape r^3 of hg_shape (r = 1/sqrt(den), den = (1-g)^2 + 2 g u) and,
// from the same denominator, d ln HG / d g = c0 - 3 (g - 1 + u) / den with
// c0 = -2g / (1 - g^2) and 1/den = r^2 (rho built from g; gm1 = g - 1).
__device__ __forceinline__ float hg_shape_dlog(const HG& rho, float c0, float gm1, f3 t, float wx, float wy,
                                               float wz, float& dl) {
    const float dx = t.x - wx, dy = t.y - wy, dz = t.z - wz;
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float r = __frsqrt_rn(fmaf(0.5f * rho.two_g, d2, rho.a));
    const float r2 = r * r;
    dl = fmaf(-3.0f * fmaf(0.5f, d2, gm1), r2, c0);
    return r2 * r;
}

// sum_j rho_i(w_j) (1/M+_j) x_j over the cluster [a, e)
__device__ __forceinline__ f3 cluster_gather(const HG& rho, f3 ti, uint2 rg, const float4* __restrict__ wq,
                                             const float* __restrict__ x) {
    float zx = 0.f, zy = 0.f, zz = 0.f;
    for (uint32_t j = rg.x; j < rg.y; ++j) {
        const float4 w4 = wq[j];
        const float f = hg_shape(rho, ti, w4.x, w4.y, w4.z) * w4.w;
        const f3 xv = ld3(x, j);
        zx = fmaf(f, xv.x, zx);
        zy = fmaf(f, xv.y, zy);
        zz = fmaf(f, xv.z, zz);
    }
    return f3{zx, zy, zz};
}

// y_i = b_i + alpha_i sum_j w+_ij x_j, the weights recomputed; one thread
// per row.  The clusters of a block's rows cover one contiguous span of
// positions (its rows plus the parts of the first and last cluster outside
// the block); when the span fits kSpan, the members' (w, 1/M+) and x are
// staged in LDS once, with coalesced loads, and every row sums from there.
//
// With SHIFTED the propagation is folded in: x is not stored, the members'
// values are gathered as x_j = y_prev(succ j) (0 at a path's end), so one
// launch per iteration replaces the aggregation and the shift.
constexpr int kSpan = 512;
template <bool SHIFTED>
__global__ __launch_bounds__(kBlock) void k_cagg(int64_t N, HG rho, const uint2* __restrict__ crange,
                                                 const float4* __restrict__ tq, const float4* __restrict__ wq,
                                                 const float* __restrict__ b, const float* __restrict__ x,
                                                 const int32_t* __restrict__ succ, float* __restrict__ y) {
    __shared__ float4 sw[kSpan];
    __shared__ float sx[3 * kSpan];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);   // the path neighbours' lines on one L2
    const int64_t i0 = tile * kBlock;
    const int64_t i = i0 + threadIdx.x;
    const int64_t ilast = i0 + kBlock - 1 < N ? i0 + kBlock - 1 : N - 1;
    const uint32_t lo = crange[i0].x, hi = crange[ilast].y;
    const bool staged = hi - lo <= (uint32_t)kSpan;   // uniform over the block
    if (staged) {
        for (uint32_t t = threadIdx.x; t < hi - lo; t += kBlock) {
            sw[t] = wq[lo + t];
            if (SHIFTED) {
                const int32_t sj = __builtin_nontemporal_load(succ + lo + t);
                const f3 v = sj >= 0 ? ld3(x, sj) : f3{0.f, 0.f, 0.f};
                sx[3 * t] = v.x;
                sx[3 * t + 1] = v.y;
                sx[3 * t + 2] = v.z;
            }
        }
        if (!SHIFTED)
            for (uint32_t t = threadIdx.x; t < 3 * (hi - lo); t += kBlock) sx[t] = x[3 * (int64_t)lo + t];
        __syncthreads();
    }
    if (i >= N) return;
    const float4 t4 = tq[i];
    const f3 ti{t4.x, t4.y, t4.z};
    const uint2 rg = bounded(crange[i]);
    f3 z;
    if (staged) {
        float zx = 0.f, zy = 0.f, zz = 0.f;
        for (uint32_t j = rg.x - lo; j < rg.y - lo; ++j) {
            const float4 w4 = sw[j];
            const float f = hg_shape(rho, ti, w4.x, w4.y, w4.z) * w4.w;
            zx = fmaf(f, sx[3 * j], zx);
            zy = fmaf(f, sx[3 * j + 1], zy);
            zz = fmaf(f, sx[3 * j + 2], zz);
        }
        z = f3{zx, zy, zz};
    } else if (SHIFTED) {
        float zx = 0.f, zy = 0.f, zz = 0.f;
        for (uint32_t j = rg.x; j < rg.y; ++j) {
            const float4 w4 = wq[j];
            const float f = hg_shape(rho, ti, w4.x, w4.y, w4.z) * w4.w;
            const int32_t sj = succ[j];
            const f3 xv = sj >= 0 ? ld3(x, sj) : f3{0.f, 0.f, 0.f};
            zx = fmaf(f, xv.x, zx);
            zy = fmaf(f, xv.y, zy);
            zz = fmaf(f, xv.z, zz);
        }
        z = f3{zx, zy, zz};
    } else {
        z = cluster_gather(rho, ti, rg, wq, x);
    }
    const f3 bb = ld3(b, i);
    st3_nt(y, i, f3{fmaf(t4.w, z.x, bb.x), fmaf(t4.w, z.y, bb.y), fmaf(t4.w, z.z, bb.z)});
}

// One thread per pixel, as the sliced-ELL output but gathering over the
// first vertex's cluster.
__global__ __launch_bounds__(kBlock) void k_cpixels(pg_paths P, Consts c, const int32_t* __restrict__ cinv,
                                                    const uint2* __restrict__ crange, const float4* __restrict__ tq,
                                                    const float4* __restrict__ wq, const float* __restrict__ x,
                                                    const float* __restrict__ dpt, const float* __restrict__ r,
                                                    float* __restrict__ image) {
    const int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)P.width * P.height;
    if (px >= npix) return;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int k = 0; k < P.spp; ++k) {
        const int64_t p = px * P.spp + k;
        sx += P.e_cam[3 * p];
        sy += P.e_cam[3 * p + 1];
        sz += P.e_cam[3 * p + 2];
        const int64_t a = P.path_offsets[p], e = P.path_offsets[p + 1];
        if (e <= a || a < 0 || e > P.n_vertices) continue;
        const int64_t i = cinv[a];
        const float4 t4 = tq[i];
        f3 in;
        if (c.final_gather == 0) {
            in = cluster_gather(c.rho, f3{t4.x, t4.y, t4.z}, bounded(crange[i]), wq, x);
        } else {
            const float rr = r[i];
            in = f3{rr * x[3 * i], rr * x[3 * i + 1], rr * x[3 * i + 2]};
        }
        if (P.l_emit) {
            sx += P.l_emit[3 * a];
            sy += P.l_emit[3 * a + 1];
            sz += P.l_emit[3 * a + 2];
        }
        f3 dd = ld3(dpt, i);
        if (P.n_extra > 0) dd = extra_direct(P, p, a, f3{t4.x, t4.y, t4.z}, c.rho, c.g, c.sun, c.env_pdf, nullptr);
        sx = fmaf(t4.w, dd.x + in.x, sx);
        sy = fmaf(t4.w, dd.y + in.y, sy);
        sz = fmaf(t4.w, dd.z + in.z, sz);
    }
    const float inv_spp = 1.0f / (float)P.spp;
    image[3 * px] = sx * inv_spp;
    image[3 * px + 1] = sy * inv_spp;
    image[3 * px + 2] = sz * inv_spp;
}

// ---------------------------------------------------------- the export ---

// Row lengths (path order) and one partial sum of them per block, in 64 bits.
__global__ __launch_bounds__(kBlock) void k_crow_len(int64_t N, const int32_t* __restrict__ cinv,
                                                     const uint2* __restrict__ crange, uint32_t* __restrict__ len,
                                                     unsigned long long* __restrict__ part) {
    __shared__ unsigned long long sm[kBlock / kWave];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long e = 0;
    if (v < N) {
        const uint2 rg = crange[cinv[v]];
        len[v] = rg.y - rg.x;
        e = rg.y - rg.x;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) e += __shfl_xor(e, o, kWave);
    if (__lane_id() == 0) sm[threadIdx.x / kWave] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) e += sm[w];
        part[blockIdx.x] = e;
    }
}

__global__ __launch_bounds__(1024) void k_sum_final(int64_t n, const unsigned long long* __restrict__ part,
                                                    unsigned long long* __restrict__ total) {
    __shared__ unsigned long long sm[1024 / kWave];
    unsigned long long e = 0;
    for (int64_t t = threadIdx.x; t < n; t += 1024) e += part[t];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) e += __shfl_xor(e, o, kWave);
    if (__lane_id() == 0) sm[threadIdx.x / kWave] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / kWave; ++w) e += sm[w];
        *total = e;
    }
}

// Row v (path order) of the exported CSR: its cluster's members, ascending
// path id, with the three weights.  Writes nothing if the edges exceed the
// caller's capacity or 2^32.
__global__ __launch_bounds__(kBlock) void k_cexport(int64_t N, Consts c, const uint32_t* __restrict__ start,
                                                    const unsigned long long* __restrict__ nedge, int64_t capacity,
                                                    const int32_t* __restrict__ cinv, const uint2* __restrict__ crange,
                                                    const int32_t* __restrict__ cperm,
                                                    const int32_t* __restrict__ perm, const VRec* __restrict__ crec,
                                                    const float4* __restrict__ tq, const float4* __restrict__ wq,
                                                    const float* __restrict__ mp, const float* __restrict__ me,
                                                    int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                    float* __restrict__ w_ind, float* __restrict__ w_ph,
                                                    float* __restrict__ w_env, int32_t* flag) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long E = *nedge;
    const bool fits = E <= (unsigned long long)capacity && E < (1ull << 32);
    if (v == 0 && !fits) set_flag(flag, kFlagCapacity);
    if (v > N) return;
    if (row_ptr) row_ptr[v] = v == N ? (int64_t)E : (int64_t)start[v];
    if (v == N || !fits || !col) return;
    const int64_t i = cinv[v];
    const uint2 rg = bounded(crange[i]);
    const float4 t4 = tq[i];
    const f3 ti{t4.x, t4.y, t4.z};
    const int64_t base = start[v];
    for (uint32_t j = rg.x; j < rg.y; ++j) {
        const int64_t e = base + (j - rg.x);
        col[e] = perm[cperm[j]];
        const float4 w4 = wq[j];
        const float rho = c.rho(one_minus_cos(ti, f3{w4.x, w4.y, w4.z}));
        if (w_ind) w_ind[e] = hg_shape(c.rho, ti, w4.x, w4.y, w4.z) * w4.w;
        if (w_ph) w_ph[e] = rho / mp[j];
        if (w_env) {
            const VRec& rj = crec[j];
            w_env[e] = c.rho(one_minus_cos(ti, f3{rj.we[0], rj.we[1], rj.we[2]})) / me[j];
        }
    }
}

// ------------------------------------------------------- reverse mode ---
// The adjoint of the cluster render, in cluster order.  The tape holds
// x_0 (traj[0]) and y_1..y_D (traj[t]): L_{t-1}(j) = x_0(j) for t = 1, else
// y_{t-1}(succ j).  W_ij = rho_i(w_j) c_g / M+_j inside a cluster; since a
// sample's cluster is also its receivers' cluster, the transpose product
// lam_{t-1}(j) = sum_i W_ij zbar_i runs over the same member range as the
// forward product, with the roles of (t, w) swapped: no transpose is built.

// L_{t-1}(j) of the tape
template <bool SHIFTED>
__device__ __forceinline__ f3 tape_x(const float* __restrict__ x, const int32_t* __restrict__ succ, int64_t j) {
    if (!SHIFTED) return ld3(x, j);
    const int32_t sj = succ[j];
    return sj >= 0 ? ld3(x, sj) : f3{0.f, 0.f, 0.f};
}

// Output: o_p = e + alpha (d + in) at the first vertex i of path p.
__global__ __launch_bounds__(kBlock) void k_cout_adjoint(pg_paths P, Consts c, const int32_t* __restrict__ cinv,
                                                         const uint2* __restrict__ crange,
                                                         const float4* __restrict__ tq, const float4* __restrict__ wq,
                                                         const float* __restrict__ xD, const float* __restrict__ dpt,
                                                         const float* __restrict__ r, const float* __restrict__ gimg,
                                                         float* __restrict__ abar, float* __restrict__ dptbar,
                                                         float* __restrict__ rbar, float* __restrict__ lam,
                                                         double* __restrict__ gpart) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gl = 0.0;
    if (p < P.n_paths) {
        const int64_t a = P.path_offsets[p], e = P.path_offsets[p + 1];
        if (e > a && a >= 0 && e <= P.n_vertices) {
            const int64_t px = p / P.spp, i = cinv[a];
            const float is = 1.0f / (float)P.spp;
            const f3 ob{gimg[3 * px] * is, gimg[3 * px + 1] * is, gimg[3 * px + 2] * is};
            const float4 t4 = tq[i];
            const f3 ti{t4.x, t4.y, t4.z};
            const bool extra = P.n_extra > 0;
            f3 ddg{0.f, 0.f, 0.f};
            const f3 d = extra ? extra_direct(P, p, a, ti, c.rho, c.g, c.sun, c.env_pdf, &ddg) : ld3(dpt, i);
            const f3 zb{t4.w * ob.x, t4.w * ob.y, t4.w * ob.z};
            if (extra) gl += (double)dot3(zb, ddg);
            if (c.final_gather == 0) {
                const uint2 rg = bounded(crange[i]);
                f3 in{0.f, 0.f, 0.f}, ing{0.f, 0.f, 0.f};
                for (uint32_t j = rg.x; j < rg.y; ++j) {
                    const float4 w4 = wq[j];
                    const f3 wj{w4.x, w4.y, w4.z};
                    const float f = hg_shape(c.rho, ti, w4.x, w4.y, w4.z) * w4.w;
                    const float fh = f * hg_dlog(c.g, one_minus_cos(ti, wj));
                    const f3 xv = ld3(xD, j);
                    in = f3{fmaf(f, xv.x, in.x), fmaf(f, xv.y, in.y), fmaf(f, xv.z, in.z)};
                    ing = f3{fmaf(fh, xv.x, ing.x), fmaf(fh, xv.y, ing.y), fmaf(fh, xv.z, ing.z)};
                    atomicAdd(&lam[3 * j], f * zb.x);
                    atomicAdd(&lam[3 * j + 1], f * zb.y);
                    atomicAdd(&lam[3 * j + 2], f * zb.z);
                }
                abar[i] += dot3(ob, f3{d.x + in.x, d.y + in.y, d.z + in.z});
                gl += (double)dot3(zb, ing);
            } else {
                const f3 xv = ld3(xD, i);
                const float rr = r[i];
                abar[i] += dot3(ob, f3{fmaf(rr, xv.x, d.x), fmaf(rr, xv.y, d.y), fmaf(rr, xv.z, d.z)});
                rbar[i] += dot3(zb, xv);
                atomicAdd(&lam[3 * i], rr * zb.x);
                atomicAdd(&lam[3 * i + 1], rr * zb.y);
                atomicAdd(&lam[3 * i + 2], rr * zb.z);
            }
            if (!extra) {
                dptbar[3 * i] += zb.x;
                dptbar[3 * i + 1] += zb.y;
                dptbar[3 * i + 2] += zb.z;
            }
        }
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[blockIdx.x] = t;
}

// Row i of iteration t: y_i = b_i + alpha_i z_i, z_i = sum_j W_ij L_{t-1}(j).
// The adjoint of y_i is lam_t(pred i); adds <ybar, z_i> to abar_i and ybar to
// bbar_i, stores zbar_i = alpha_i ybar and adds <zbar_i, sum_j dW_ij/dg
// L_{t-1}(j)> (dW/dg = W h) to the block's dL/dg slot.  The block's member
// span is staged in LDS as in the forward product.
template <bool SHIFTED>
__global__ __launch_bounds__(kBlock) void k_crev_rows(int64_t N, HG rho, float g, const uint2* __restrict__ crange,
                                                      const float4* __restrict__ tq, const float4* __restrict__ wq,
                                                      const float* __restrict__ x, const int32_t* __restrict__ succ,
                                                      const float* __restrict__ lam, const int32_t* __restrict__ pred,
                                                      float* __restrict__ abar, float* __restrict__ bbar,
                                                      float* __restrict__ zbar, double* __restrict__ gpart) {
    __shared__ float4 sw[kSpan];
    __shared__ float sx[3 * kSpan];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);   // the path neighbours' lines on one L2
    const int64_t i0 = tile * kBlock;
    const int64_t i = i0 + threadIdx.x;
    const int64_t ilast = i0 + kBlock - 1 < N ? i0 + kBlock - 1 : N - 1;
    const uint32_t lo = crange[i0].x, hi = crange[ilast].y;
    const bool staged = hi - lo <= (uint32_t)kSpan;
    if (staged) {
        for (uint32_t t = threadIdx.x; t < hi - lo; t += kBlock) {
            sw[t] = wq[lo + t];
            const f3 v = tape_x<SHIFTED>(x, succ, lo + t);
            sx[3 * t] = v.x;
            sx[3 * t + 1] = v.y;
            sx[3 * t + 2] = v.z;
        }
        __syncthreads();
    }
    double gl = 0.0;
    if (i < N) {
        const float4 t4 = tq[i];
        const f3 ti{t4.x, t4.y, t4.z};
        const uint2 rg = bounded(crange[i]);
        const float c0 = -2.0f * g / (1.0f - g * g), gm1 = g - 1.0f;
        f3 z{0.f, 0.f, 0.f}, zg{0.f, 0.f, 0.f};
        for (uint32_t j = rg.x; j < rg.y; ++j) {
            const float4 w4 = staged ? sw[j - lo] : wq[j];
            const f3 xv = staged ? f3{sx[3 * (j - lo)], sx[3 * (j - lo) + 1], sx[3 * (j - lo) + 2]}
                                 : tape_x<SHIFTED>(x, succ, j);
            float dl;
            const float f = hg_shape_dlog(rho, c0, gm1, ti, w4.x, w4.y, w4.z, dl) * w4.w;
            const float fh = f * dl;
            z = f3{fmaf(f, xv.x, z.x), fmaf(f, xv.y, z.y), fmaf(f, xv.z, z.z)};
            zg = f3{fmaf(fh, xv.x, zg.x), fmaf(fh, xv.y, zg.y), fmaf(fh, xv.z, zg.z)};
        }
        const int32_t pv = pred[i];
        const f3 yb = pv >= 0 ? ld3(lam, pv) : f3{0.f, 0.f, 0.f};
        abar[i] += dot3(yb, z);
        bbar[3 * i] += yb.x;
        bbar[3 * i + 1] += yb.y;
        bbar[3 * i + 2] += yb.z;
        const f3 zb{t4.w * yb.x, t4.w * yb.y, t4.w * yb.z};
        st3(zbar, i, zb);
        gl = (double)dot3(zb, zg);
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[tile] += t;
}

// lam_{t-1}(j) = sum_{i in cluster(j)} W_ij zbar_i = (c_g / M+_j) sum_i
// rho_i(w_j) zbar_i: the receivers' (t_i, zbar_i) of the span in LDS.
__global__ __launch_bounds__(kBlock) void k_crev_cols(int64_t N, HG rho, const uint2* __restrict__ crange,
                                                      const float4* __restrict__ tq, const float4* __restrict__ wq,
                                                      const float* __restrict__ zbar, float* __restrict__ lam) {
    __shared__ float4 st[kSpan];
    __shared__ float sz[3 * kSpan];
    const int64_t j0 = (int64_t)blockIdx.x * kBlock;
    const int64_t j = j0 + threadIdx.x;
    const int64_t jlast = j0 + kBlock - 1 < N ? j0 + kBlock - 1 : N - 1;
    const uint32_t lo = crange[j0].x, hi = crange[jlast].y;
    const bool staged = hi - lo <= (uint32_t)kSpan;
    if (staged) {
        for (uint32_t t = threadIdx.x; t < hi - lo; t += kBlock) st[t] = tq[lo + t];
        for (uint32_t t = threadIdx.x; t < 3 * (hi - lo); t += kBlock) sz[t] = zbar[3 * (int64_t)lo + t];
        __syncthreads();
    }
    if (j >= N) return;
    const float4 w4 = wq[j];
    const uint2 rg = bounded(crange[j]);
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (uint32_t i = rg.x; i < rg.y; ++i) {
        const float4 t4 = staged ? st[i - lo] : tq[i];
        const f3 zb = staged ? f3{sz[3 * (i - lo)], sz[3 * (i - lo) + 1], sz[3 * (i - lo) + 2]} : ld3(zbar, i);
        const float f = hg_shape(rho, f3{t4.x, t4.y, t4.z}, w4.x, w4.y, w4.z);
        ax = fmaf(f, zb.x, ax);
        ay = fmaf(f, zb.y, ay);
        az = fmaf(f, zb.z, az);
    }
    st3(lam, j, f3{ax * w4.w, ay * w4.w, az * w4.w});
}

// Direct terms, per receiver over its cluster (mirrors k_cedges):
//   d/d alpha_i += <bbar_i, d_agg_i>,
//   dL/dg += <alpha_i bbar_i, d d_agg_i/dg> + <dptbar_i, d d_pt_i/dg> + rbar_i r_i h(u_w,i).
__global__ __launch_bounds__(kBlock) void k_cedges_adjoint(int64_t N, Consts c, const uint2* __restrict__ crange,
                                                           const VRec* __restrict__ crec,
                                                           const float4* __restrict__ tq,
                                                           const float* __restrict__ mp, const float* __restrict__ me,
                                                           const int32_t* __restrict__ cpid,
                                                           const float* __restrict__ dir_pl,
                                                           const float* __restrict__ l_pl,
                                                           const float* __restrict__ bbar,
                                                           const float* __restrict__ dptbar,
                                                           const float* __restrict__ rbar, float* __restrict__ abar,
                                                           double* __restrict__ gpart) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gl = 0.0;
    if (i < N) {
        const uint2 rg = bounded(crange[i]);
        const float4 t4 = tq[i];
        const f3 ti{t4.x, t4.y, t4.z};
        f3 cv{0.f, 0.f, 0.f}, ch{0.f, 0.f, 0.f}, sv{0.f, 0.f, 0.f}, qv{0.f, 0.f, 0.f}, qh{0.f, 0.f, 0.f};
        for (uint32_t j = rg.x; j < rg.y; ++j) {
            const VRec& rj = crec[j];
            const f3 wj{rj.w[0], rj.w[1], rj.w[2]}, wej{rj.we[0], rj.we[1], rj.we[2]};
            const float uw = one_minus_cos(ti, wj), ue = one_minus_cos(ti, wej);
            const float fp = c.rho(uw) / mp[j], fe = c.rho(ue) / me[j];
            const float hp = hg_dlog(c.g, uw), he = hg_dlog(c.g, ue);
            for (int a = 0; a < 3; ++a) {
                const float v = fe * rj.le[a] + fp * rj.lp[a], h = fe * he * rj.le[a] + fp * hp * rj.lp[a];
                if (a == 0) { cv.x += v; ch.x += h; sv.x += rj.ls[0]; }
                if (a == 1) { cv.y += v; ch.y += h; sv.y += rj.ls[1]; }
                if (a == 2) { cv.z += v; ch.z += h; sv.z += rj.ls[2]; }
            }
            if (dir_pl) {
                const int64_t pj = cpid[j];
                const float u = one_minus_cos(ti, ld3(dir_pl, pj));
                const float rpl = c.rho(u), hpl = rpl * hg_dlog(c.g, u);
                const f3 lq = ld3(l_pl, pj);
                qv = f3{fmaf(rpl, lq.x, qv.x), fmaf(rpl, lq.y, qv.y), fmaf(rpl, lq.z, qv.z)};
                qh = f3{fmaf(hpl, lq.x, qh.x), fmaf(hpl, lq.y, qh.y), fmaf(hpl, lq.z, qh.z)};
            }
        }
        const float us = one_minus_cos(ti, c.sun);
        const float rho_sun = c.rho(us), hs = hg_dlog(c.g, us);
        const float invC = 1.0f / (float)(rg.y - rg.x);
        const f3 dagg{fmaf(rho_sun * invC, sv.x, fmaf(invC, qv.x, cv.x)),
                      fmaf(rho_sun * invC, sv.y, fmaf(invC, qv.y, cv.y)),
                      fmaf(rho_sun * invC, sv.z, fmaf(invC, qv.z, cv.z))};
        const f3 bb = ld3(bbar, i);
        abar[i] += dot3(bb, dagg);
        const f3 db{t4.w * bb.x, t4.w * bb.y, t4.w * bb.z};
        const float ks = rho_sun * hs * invC;
        gl += (double)dot3(db, f3{fmaf(ks, sv.x, fmaf(invC, qh.x, ch.x)), fmaf(ks, sv.y, fmaf(invC, qh.y, ch.y)),
                                  fmaf(ks, sv.z, fmaf(invC, qh.z, ch.z))});
        // own direct term and continuation ratio
        const VRec& ri = crec[i];
        const f3 w{ri.w[0], ri.w[1], ri.w[2]}, we{ri.we[0], ri.we[1], ri.we[2]};
        const float u_w = one_minus_cos(ti, w), u_e = one_minus_cos(ti, we);
        const float rho = c.rho(u_w), rho_e = c.rho(u_e);
        const float hw = hg_dlog(c.g, u_w), he = hg_dlog(c.g, u_e);
        const float p_w = c.pdf(u_w), p_e = c.pdf(u_e);
        const float f_env = rho_e / (p_e + c.env_pdf), f_out = rho / (p_w + c.env_pdf);
        const f3 pb = ld3(dptbar, i);
        f3 dd{rho_sun * hs * ri.ls[0] + f_env * he * ri.le[0] + f_out * hw * ri.lp[0],
              rho_sun * hs * ri.ls[1] + f_env * he * ri.le[1] + f_out * hw * ri.lp[1],
              rho_sun * hs * ri.ls[2] + f_env * he * ri.le[2] + f_out * hw * ri.lp[2]};
        if (dir_pl) {
            const int64_t pi = cpid[i];
            const float u = one_minus_cos(ti, ld3(dir_pl, pi));
            const float hpl = c.rho(u) * hg_dlog(c.g, u);
            const f3 lq = ld3(l_pl, pi);
            dd = f3{fmaf(hpl, lq.x, dd.x), fmaf(hpl, lq.y, dd.y), fmaf(hpl, lq.z, dd.z)};
        }
        gl += (double)dot3(pb, dd);
        gl += (double)(rbar[i] * (rho / p_w) * hw);
    }
    const double t = block_sum_d(gl);
    if (threadIdx.x == 0) gpart[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_cpid(int64_t N, const int32_t* __restrict__ cperm,
                                                 const int32_t* __restrict__ perm, int32_t* __restrict__ cpid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) cpid[i] = perm[cperm[i]];
}

}  // namespace

int cluster_grid_bits(int64_t N, int K) {
    const double m = (double)(N / (K > 0 ? K : 1));
    int b = m > 1.0 ? (int)std::lround(std::log2(m) / 3.0) : 0;
    return b < 0 ? 0 : (b > 9 ? 9 : b);
}

void carve_clusters(Carver& cv, ClusterBufs& cb, int64_t N, int K) {
    cb.K = K;
    cb.bits = cluster_grid_bits(N, K);
    cb.ncells = (int64_t)1 << (3 * cb.bits);
    cb.kmin = cv.take<unsigned long long>(32);
    cb.nedge = cv.take<unsigned long long>(32);
    cb.part = cv.take<unsigned long long>(div_up(N, kBlock) + 1);
    cb.live = cv.take<int32_t>(64);   // [0] = 1, [1 + r] = a cluster was split in round r
    cb.gcount = cv.take<uint32_t>(cb.ncells + 1);
    cb.gpart = cv.take<uint32_t>(scan_partials_bytes(cb.ncells + 1) / 4);
    cb.gcell = cv.take<uint32_t>(N);
    cb.grank = cv.take<uint32_t>(N);
    cb.gq = cv.take<uint64_t>(N);
    cb.gs = cv.take<int32_t>(N);
    cb.gpid = cv.take<int32_t>(N);
    cb.cid = cv.take<int32_t>(N);
    cb.ccount = cv.take<uint32_t>(N + 1);
    cb.cstart = cv.take<uint32_t>(N + 1);
    cb.cpart = cv.take<uint32_t>(scan_partials_bytes(N + 1) / 4);
    cb.cfill = cv.take<uint32_t>(N);
    cb.members = cv.take<int32_t>(N);
    cb.mslot = cv.take<uint32_t>(N);
    cb.mkey = cv.take<unsigned long long>(N);
    cb.mq = cv.take<uint64_t>(N);
    cb.newc = cv.take<uint8_t>(N);
    cb.nsplit = cv.take<uint32_t>(kClusterRounds);
    cb.splitlist = cv.take<int32_t>(N / (2 * (int64_t)K + 1) + 1);
    cb.stage_m = cv.take<int32_t>(N);
    cb.stage_k = cv.take<unsigned long long>(N);
    cb.stage_q = cv.take<uint64_t>(N);
    cb.cperm = cv.take<int32_t>(N);
    cb.cinv = cv.take<int32_t>(N);
    cb.crange = cv.take<uint2>(N);
}

#define PG_TRY(x)                              \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

static dim3 grid_of(int64_t n) { return dim3((unsigned)div_up(n > 0 ? n : 1, kBlock)); }

// Groups the vertices by cluster (counts, starts, members): once, after the
// nearest-centre assignment; the split rounds then regroup in place.
static hipError_t group(const pg_paths* p, const GridBufs& g, int64_t N, ClusterBufs& cb, hipStream_t s) {
    PG_TRY(launch_fill(cb.ccount, (size_t)(N + 1) * 4, s));
    PG_TRY(launch_fill(cb.cfill, (size_t)N * 4, s));
    hipLaunchKernelGGL(k_ccount, grid_of(N), dim3(kBlock), 0, s, N, cb.cid, cb.ccount);
    PG_TRY(hipGetLastError());
    PG_TRY(launch_scan_exclusive(cb.ccount, cb.cstart, N + 1, cb.cpart, s));
    hipLaunchKernelGGL(k_cgroup, grid_of(N), dim3(kBlock), 0, s, N, cb.cid, cb.cstart, cb.cfill, g.perm,
                       p->cluster_key, g.qs, cb.members, cb.mslot, cb.mkey, cb.mq);
    return hipGetLastError();
}

hipError_t run_clusters(const pg_paths* p, GridBufs& g, ClusterBufs& cb, hipStream_t s) {
    const int64_t N = p->n_vertices;
    const int K = cb.K;
    PG_TRY(launch_fill(cb.nedge, 8, s));
    if (N == 0) return hipSuccess;
    PG_TRY(launch_fill(cb.live, 64 * 4, s));
    PG_TRY(launch_fill_value(cb.live, 4, 1u, s));
    PG_TRY(launch_fill(cb.nsplit, kClusterRounds * 4, s));
    const int64_t nb = div_up(N, kBlock);
    hipLaunchKernelGGL(k_key_min, dim3((unsigned)nb), dim3(kBlock), 0, s, N, p->cluster_key, cb.part);
    PG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_key_min_final, dim3(1), dim3(1024), 0, s, nb, cb.part, cb.kmin);
    PG_TRY(hipGetLastError());
    const unsigned long long thr = (1ull << 32) / (unsigned long long)K;
    // uniform grid of the centres
    PG_TRY(launch_fill(cb.gcount, (size_t)(cb.ncells + 1) * 4, s));
    hipLaunchKernelGGL(k_cg_count, grid_of(N), dim3(kBlock), 0, s, N, g.perm, p->cluster_key, thr, cb.kmin, g.qs,
                       cb.bits, cb.gcount, cb.gcell, cb.grank);
    PG_TRY(hipGetLastError());
    PG_TRY(launch_scan_exclusive(cb.gcount, cb.gcount, cb.ncells + 1, cb.gpart, s));
    hipLaunchKernelGGL(k_cg_scatter, grid_of(N), dim3(kBlock), 0, s, N, g.perm, p->cluster_key, thr, cb.kmin, g.qs,
                       cb.gcell, cb.grank, cb.gcount, cb.gq, cb.gs, cb.gpid);
    PG_TRY(hipGetLastError());
    {
        ProfScope ps(s, "nearest_centre");
        hipLaunchKernelGGL(k_nearest_centre, grid_of(N), dim3(kBlock), 0, s, N, g.qs, cb.bits, cb.gcount, cb.gq,
                           cb.gs, cb.gpid, cb.cid, g.flag);
        PG_TRY(hipGetLastError());
    }
    // split rounds; round r runs only if round r-1 split something.  The
    // vertices are grouped by centre once; a round regroups only the
    // clusters it split, each inside its own range.
    {
        ProfScope ps(s, "split");
        PG_TRY(group(p, g, N, cb, s));
        const unsigned rg_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, N / (2 * (int64_t)K + 1)));
        for (int r = 0; r < kClusterRounds; ++r) {
            const int32_t* live = cb.live + r;
            hipLaunchKernelGGL(k_split_mark, grid_of(N), dim3(kBlock), 0, s, N, K, cb.cid, cb.ccount, cb.cstart,
                               cb.mslot, cb.mkey, cb.newc, live, cb.live + r + 1, cb.nsplit + r, cb.splitlist,
                               g.flag);
            PG_TRY(hipGetLastError());
            hipLaunchKernelGGL(k_split_assign, grid_of(N), dim3(kBlock), 0, s, N, K, g.qs, cb.cid, cb.ccount,
                               cb.cstart, cb.members, cb.mkey, cb.mq, cb.newc, live);
            PG_TRY(hipGetLastError());
            hipLaunchKernelGGL(k_regroup, dim3(rg_blocks), dim3(kBlock), 0, s, cb.splitlist, cb.nsplit + r, cb.cid,
                               cb.ccount, cb.cstart, cb.members, cb.mslot, cb.mkey, cb.mq, cb.newc, cb.stage_m,
                               cb.stage_k, cb.stage_q);
            PG_TRY(hipGetLastError());
        }
    }
    ProfScope ps(s, "cluster_order");
    hipLaunchKernelGGL(k_corder, grid_of(N), dim3(kBlock), 0, s, N, cb.cid, cb.ccount, cb.cstart, cb.mslot,
                       cb.mkey, g.perm, cb.cperm, cb.cinv, cb.crange, g.flag);
    return hipGetLastError();
}

// Path id of each vertex's cluster centre, path order.
__global__ __launch_bounds__(kBlock) void k_centre_out(int64_t N, const int32_t* __restrict__ inv,
                                                       const int32_t* __restrict__ cid,
                                                       const int32_t* __restrict__ perm, int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) out[v] = perm[cid[inv[v]]];
}

hipError_t launch_centre_out(int64_t N, const GridBufs& g, const ClusterBufs& cb, int32_t* out, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_centre_out, grid_of(N), dim3(kBlock), 0, s, N, g.inv, cb.cid, g.perm, out);
    return hipGetLastError();
}

// ------------------------------------------------------ cluster render ---

void carve_cluster_render(Carver& cv, ClusterRender& cr, int64_t N) {
    cr.crec = cv.take<VRec>(N);
    cr.tq = cv.take<float4>(N);
    cr.wq = cv.take<float4>(N);
    cr.mp = cv.take<float>(N);
    cr.me = cv.take<float>(N);
    cr.y2 = cv.take<float>(3 * N);
    cr.rowlen = cv.take<uint32_t>(N + 1);
    cr.rowpart = cv.take<uint32_t>(scan_partials_bytes(N + 1) / 4);
}

hipError_t cluster_setup(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                         hipStream_t s, float** x0_out) {
    const int64_t N = r.N;
    GridBufs& g = r.g;
    ClusterBufs& cb = r.cl;
    ClusterRender& cr = r.cr;
    {
        ProfScope ps(s, "grid");
        PG_TRY(run_grid(p, g, r.rec, s));
    }
    PG_TRY(run_clusters(p, g, cb, s));
    const Consts c = make_consts(q, r.K);
    if (N > 0) {
        ProfScope ps(s, "edges");
        hipLaunchKernelGGL(k_crec, grid_of(N), dim3(kBlock), 0, s, N, cb.cperm, r.rec, cr.crec, cr.tq, r.alpha);
        PG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_cmarg, grid_of(N), dim3(kBlock), 0, s, N, c, cb.crange, cr.crec, cr.tq, cr.wq, cr.mp,
                           cr.me);
        PG_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_cedges, grid_of(N), dim3(kBlock), 0, s, N, c, cb.crange, cr.crec, cr.tq, cr.mp, cr.me,
                           p->l_emit, cb.cperm, g.perm, p->dir_pl, p->l_pl, r.b, r.dpt, r.r);
        PG_TRY(hipGetLastError());
    }
    if (out && (out->row_ptr || out->col)) {
        hipLaunchKernelGGL(k_crow_len, grid_of(N), dim3(kBlock), 0, s, N, cb.cinv, cb.crange, cr.rowlen, cb.part);
        PG_TRY(hipGetLastError());
        if (N > 0) {
            hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(1024), 0, s, div_up(N, kBlock), cb.part, cb.nedge);
            PG_TRY(hipGetLastError());
        }
        PG_TRY(launch_fill(cr.rowlen + N, 4, s));
        PG_TRY(launch_scan_exclusive(cr.rowlen, cr.rowlen, N + 1, cr.rowpart, s));
        hipLaunchKernelGGL(k_cexport, grid_of(N + 1), dim3(kBlock), 0, s, N, c, cr.rowlen, cb.nedge,
                           out->edge_capacity, cb.cinv, cb.crange, cb.cperm, g.perm, cr.crec, cr.tq, cr.wq, cr.mp,
                           cr.me, out->row_ptr, out->col, out->w_ind, out->w_ph, out->w_env, g.flag);
        PG_TRY(hipGetLastError());
    }
    if (out && out->b) PG_TRY(launch_permute3(N, cb.cinv, r.b, out->b, 1, s));
    if (out && out->d_pt) PG_TRY(launch_permute3(N, cb.cinv, r.dpt, out->d_pt, 1, s));
    float* x0 = r.tape ? r.traj : r.x;   // with the tape, traj[0] = x_0 and traj[t] = y_t
    PG_TRY(launch_fill_value(r.succ, (size_t)N * 4, 0xffffffffu, s));
    if (r.pred) PG_TRY(launch_fill_value(r.pred, (size_t)N * 4, 0xffffffffu, s));
    PG_TRY(launch_fill(x0, (size_t)N * 12, s));
    {
        ProfScope ps(s, "paths");
        PG_TRY(launch_paths(r.P, N, p->path_offsets, cb.cinv, r.alpha, r.dpt, r.r, p->l_emit, q->init, r.succ,
                            r.pred, x0, g.flag, s));
    }
    *x0_out = x0;
    return hipSuccess;
}

// Iteration 1 aggregates the stored L_0; iterations 2..D gather L_{t-1} =
// y_{t-1}(succ) inside the aggregation (y ping-pongs between y and x); one
// shift at the end materialises L_D.
hipError_t cluster_iterate(RenderBufs& r, const pg_params* q, float* x0, hipStream_t s, float** final_x) {
    const int64_t N = r.N;
    const HG rho = HG::make(q->g);
    if (r.D == 0 || N == 0) {
        *final_x = x0;
        return hipSuccess;
    }
    float* yp = r.tape ? r.traj + (size_t)N * 3 : r.y;   // y_1
    float* yq = r.cr.y2;
    for (int t = 1; t <= r.D; ++t) {
        ProfScope ps(s, "spmv");
        if (t == 1) {
            hipLaunchKernelGGL(k_cagg<false>, grid_of(N), dim3(kBlock), 0, s, N, rho, r.cl.crange, r.cr.tq, r.cr.wq,
                               r.b, x0, r.succ, yp);
        } else {
            if (r.tape) yq = r.traj + (size_t)t * N * 3;
            hipLaunchKernelGGL(k_cagg<true>, grid_of(N), dim3(kBlock), 0, s, N, rho, r.cl.crange, r.cr.tq, r.cr.wq,
                               r.b, yp, r.succ, yq);
        }
        PG_TRY(hipGetLastError());
        if (t > 1) std::swap(yp, yq);
    }
    ProfScope ps(s, "shift");
    PG_TRY(launch_shift(N, r.succ, yp, r.x, s));   // L_D (with the tape x_0 stays in traj[0])
    *final_x = r.x;
    return hipSuccess;
}

hipError_t cluster_output(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                          float* image, const float* cur, hipStream_t s) {
    const Consts c = make_consts(q, r.K);
    const int64_t npix = (int64_t)p->width * p->height;
    if (npix > 0) {
        ProfScope ps(s, "pixels");
        hipLaunchKernelGGL(k_cpixels, grid_of(npix), dim3(kBlock), 0, s, *p, c, r.cl.cinv, r.cl.crange, r.cr.tq,
                           r.cr.wq, cur, r.dpt, r.r, image);
        PG_TRY(hipGetLastError());
    }
    if (out && out->lplus) PG_TRY(launch_permute3(r.N, r.cl.cinv, cur, out->lplus, 1, s));
    if (out && out->n_far) PG_TRY(launch_fill(out->n_far, sizeof(int64_t), s));   // no compact ids here
    return hipSuccess;
}

// ------------------------------------------------ reverse-mode launchers ---

hipError_t launch_cluster_cpid(int64_t N, const RenderBufs& r, int32_t* cpid, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cpid, grid_of(N), dim3(kBlock), 0, s, N, r.cl.cperm, r.g.perm, cpid);
    return hipGetLastError();
}

hipError_t launch_cluster_out_adjoint(const pg_paths& P, const Consts& c, const RenderBufs& r, const float* gimg,
                                      float* abar, float* dptbar, float* rbar, float* lam, double* gpart,
                                      int64_t nblocks, hipStream_t s) {
    const float* xD = r.D == 0 ? r.traj : r.x;   // L_D (x_0 itself when there is no iteration)
    hipLaunchKernelGGL(k_cout_adjoint, dim3((unsigned)nblocks), dim3(kBlock), 0, s, P, c, r.cl.cinv, r.cl.crange,
                       r.cr.tq, r.cr.wq, xD, r.dpt, r.r, gimg, abar, dptbar, rbar, lam, gpart);
    return hipGetLastError();
}

// Reverse of iteration t: rows (adjoint of y_t, zbar), then columns (lam_{t-1}).
hipError_t launch_cluster_reverse_step(const RenderBufs& r, const pg_params* q, int t, const float* lam,
                                       float* lam_prev, float* abar, float* bbar, float* zbar, double* gpart,
                                       hipStream_t s) {
    const int64_t N = r.N;
    if (N == 0) return hipSuccess;
    const HG rho = HG::make(q->g);
    const float* x = r.traj + (size_t)(t - 1) * N * 3;   // x_0, or y_{t-1} to be gathered through succ
    {
        ProfScope ps(s, "rev_rows");
        if (t == 1)
            hipLaunchKernelGGL(k_crev_rows<false>, grid_of(N), dim3(kBlock), 0, s, N, rho, q->g, r.cl.crange,
                               r.cr.tq, r.cr.wq, x, r.succ, lam, r.pred, abar, bbar, zbar, gpart);
        else
            hipLaunchKernelGGL(k_crev_rows<true>, grid_of(N), dim3(kBlock), 0, s, N, rho, q->g, r.cl.crange,
                               r.cr.tq, r.cr.wq, x, r.succ, lam, r.pred, abar, bbar, zbar, gpart);
        PG_TRY(hipGetLastError());
    }
    ProfScope ps(s, "rev_cols");
    hipLaunchKernelGGL(k_crev_cols, grid_of(N), dim3(kBlock), 0, s, N, rho, r.cl.crange, r.cr.tq, r.cr.wq, zbar,
                       lam_prev);
    return hipGetLastError();
}

hipError_t launch_cluster_edges_adjoint(const pg_paths& P, const Consts& c, const RenderBufs& r, const int32_t* cpid,
                                        const float* bbar, const float* dptbar, const float* rbar, float* abar,
                                        double* gpart, hipStream_t s) {
    const int64_t N = r.N;
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cedges_adjoint, grid_of(N), dim3(kBlock), 0, s, N, c, r.cl.crange, r.cr.crec, r.cr.tq,
                       r.cr.mp, r.cr.me, cpid, P.dir_pl, P.l_pl, bbar, dptbar, rbar, abar, gpart);
    return hipGetLastError();
}

}  // namespace pg
