// pg_grid.hip -- uniform-grid build (counting sort) and exact k-nearest-
// neighbour query on quantised integer coordinates.
//
// The paper builds a hash grid over the shading points and searches the
// neighbouring bins (Sec. "Rendering System", path graph solver).  Here the
// neighbourhood of vertex i is exact: i first, then the K-1 nearest others by
// (squared distance of the 20-bit quantised positions, path-order id).
//
// Grid: cell = q >> shift per axis, G = 2^(20-shift) cells per axis.  The
// vertices are sorted by the position of their cell along the Hilbert curve,
// so neighbouring cells are close in memory (the gathers of the kNN, the
// edge weights and every propagation step stay in a small window); a table
// indexed by the cell's Morton number gives each cell's [start, end) in that
// order without re-encoding during the search.  Counting sort = atomic
// histogram (which also yields each vertex's rank inside its cell) +
// exclusive scan + scatter.  The order of vertices inside a cell is not
// deterministic; nothing downstream depends on it (every comparison breaks
// ties by path-order id).
#include "pg_internal.h"

namespace pg {

__device__ inline uint32_t quant(float x) {
    float s = floorf(x * 1048576.0f);   // exact: scaling by 2^20
    if (!(s >= 0.0f)) s = 0.0f;          // also NaN
    if (s > (float)kQMax) s = (float)kQMax;
    return (uint32_t)s;
}

__global__ __launch_bounds__(kBlock) void k_quantize_count(int64_t N, const float* __restrict__ pos, int shift,
                                                           uint32_t* __restrict__ count,
                                                           uint32_t* __restrict__ cellid,
                                                           uint32_t* __restrict__ rank, int32_t* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (!(x >= 0.0f && x <= 1.0f && y >= 0.0f && y <= 1.0f && z >= 0.0f && z <= 1.0f)) set_flag(flag, kFlagPos);
    uint32_t c = hilbert3(quant(x) >> shift, quant(y) >> shift, quant(z) >> shift, kQBits - shift);
    cellid[i] = c;
    rank[i] = atomicAdd(&count[c], 1u);
}

hipError_t launch_quantize_count(int64_t N, const float* pos, int shift, uint32_t* count, uint32_t* cellid,
                                 uint32_t* rank, int32_t* flag, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_quantize_count, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, pos, shift,
                       count, cellid, rank, flag);
    return hipGetLastError();
}

// range[m] = [start, end) of the cell with Morton number m, from the
// exclusive scan `start` of the counts in Hilbert order.
__global__ __launch_bounds__(kBlock) void k_cell_range(int64_t ncells, int shift, const uint32_t* __restrict__ start,
                                                       uint2* __restrict__ range) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ncells) return;
    const uint32_t u = (uint32_t)m;
    const uint32_t h = hilbert3(compact1by2(u), compact1by2(u >> 1), compact1by2(u >> 2), kQBits - shift);
    range[m] = make_uint2(start[h], start[h + 1]);
}

hipError_t launch_cell_range(int64_t ncells, int shift, const uint32_t* start, uint2* range, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_range, dim3((unsigned)div_up(ncells, kBlock)), dim3(kBlock), 0, s, ncells, shift,
                       start, range);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan ---
// Exclusive prefix sum of uint32 counts, out[n] = total.  Three passes:
// per-block totals, a scan of the block totals, per-block scans with offset.
// Inside a block: per-thread serial sums, a wave-level inclusive scan with
// lane shuffles, and a scan of the wave totals through LDS.

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline uint32_t wave_inclusive(uint32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan across the block of one value per thread; returns the
// thread's exclusive prefix and the block total.
__device__ inline uint32_t block_exclusive(uint32_t v, uint32_t& total) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t inc = wave_inclusive(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        uint32_t x = wsum[w];
        if (w < wid) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                        uint32_t* __restrict__ partials) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t total;
    block_exclusive(s, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// one block scans nb partials in tiles, carrying the running offset
__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t* __restrict__ partials, int64_t nb) {
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanTile) {
        int64_t i0 = base + (int64_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (i0 + k < nb) ? partials[i0 + k] : 0u;
            s += v[k];
        }
        uint32_t total;
        uint32_t ex = block_exclusive(s, total) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (i0 + k < nb) partials[i0 + k] = ex;
            ex += v[k];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n,
                                                      const uint32_t* __restrict__ partials) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t ex = block_exclusive(s, total) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    // the last element of the last block closes the prefix sum
    if (base < n && base + kScanItems >= n) out[n] = ex;
}

size_t scan_partials_bytes(int64_t n) { return (size_t)(div_up(n, kScanTile) + 1) * sizeof(uint32_t); }

hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                                 hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    int64_t nb = div_up(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, partials);
    return hipGetLastError();
}

// --------------------------------------------------------------- scatter ---

// Cell-centred trilinear albedo of a grid [R][R][R] (z, y, x).
__device__ inline float trilerp_alpha(const float* grid, int R, float px, float py, float pz) {
    uint32_t idx[8];
    float w[8];
    trilerp_corners(R, px, py, pz, idx, w);
    float a = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) a = fmaf(w[c], grid[idx[c]], a);
    return a;
}

__device__ inline void fill_record(const pg_paths& P, int64_t v, VRec& r) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.t[a] = P.dir_in[3 * v + a];
        r.w[a] = P.dir_out[3 * v + a];
        r.we[a] = P.dir_env[3 * v + a];
        r.ls[a] = P.l_sun[3 * v + a];
        r.le[a] = P.l_env[3 * v + a];
        r.lp[a] = P.l_phase[3 * v + a];
    }
    r.alpha = P.albedo_grid ? trilerp_alpha(P.albedo_grid, P.albedo_grid_res, P.pos[3 * v], P.pos[3 * v + 1],
                                            P.pos[3 * v + 2])
                            : P.albedo[v];
    r.pad = 0.0f;
}

__device__ inline void store_record(VRec* dst, const VRec& r) {
    const float4* s4 = reinterpret_cast<const float4*>(&r);
    float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int k = 0; k < 5; ++k) d4[k] = s4[k];
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t N, pg_paths P, int shift,
                                                    const uint32_t* __restrict__ cellid,
                                                    const uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ cell_start,
                                                    int32_t* __restrict__ perm, int32_t* __restrict__ inv,
                                                    uint64_t* __restrict__ qsorted, VRec* __restrict__ rec) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    (void)shift;
    int64_t s = (int64_t)cell_start[cellid[v]] + rank[v];
    perm[s] = (int32_t)v;
    inv[v] = (int32_t)s;
    qsorted[s] = qpack(quant(P.pos[3 * v]), quant(P.pos[3 * v + 1]), quant(P.pos[3 * v + 2]));
    if (rec) {
        VRec r;
        fill_record(P, v, r);
        store_record(rec + s, r);
    }
}

hipError_t launch_scatter(int64_t N, const pg_paths& paths, int shift, const uint32_t* cellid,
                          const uint32_t* rank, const uint32_t* cell_start, int32_t* perm, int32_t* inv,
                          uint64_t* qsorted, VRec* rec, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, paths, shift, cellid,
                       rank, cell_start, perm, inv, qsorted, rec);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_pack_records(int64_t N, pg_paths P, VRec* __restrict__ rec,
                                                         int32_t* flag) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    float x = P.pos[3 * v], y = P.pos[3 * v + 1], z = P.pos[3 * v + 2];
    if (!(x >= 0.0f && x <= 1.0f && y >= 0.0f && y <= 1.0f && z >= 0.0f && z <= 1.0f)) set_flag(flag, kFlagPos);
    VRec r;
    fill_record(P, v, r);
    store_record(rec + v, r);
}

__global__ __launch_bounds__(kBlock) void k_alpha(int64_t N, pg_paths P, float* __restrict__ alpha) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    alpha[v] = P.albedo_grid ? trilerp_alpha(P.albedo_grid, P.albedo_grid_res, P.pos[3 * v], P.pos[3 * v + 1],
                                             P.pos[3 * v + 2])
                             : P.albedo[v];
}

hipError_t launch_alpha(int64_t N, const pg_paths& paths, float* alpha, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, paths, alpha);
    return hipGetLastError();
}

// rec[s] = recp[perm[s]]: the records packed in path order, gathered into the
// sorted order (one 80-byte read and one coalesced 80-byte write per vertex
// instead of scattering them from path order).
__global__ __launch_bounds__(kBlock) void k_gather_records(int64_t N, const int32_t* __restrict__ perm,
                                                           const VRec* __restrict__ recp, VRec* __restrict__ rec) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const float4* src = reinterpret_cast<const float4*>(recp + perm[s]);
    float4* dst = reinterpret_cast<float4*>(rec + s);
    float4 v[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = src[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) dst[k] = v[k];
}

hipError_t launch_gather_records(int64_t N, const int32_t* perm, const VRec* recp, VRec* rec, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_records, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, perm, recp, rec);
    return hipGetLastError();
}

hipError_t launch_pack_records(int64_t N, const pg_paths& paths, VRec* rec, int32_t* flag, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_records, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, paths, rec,
                       flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------- kNN ---
// One query per thread, queries in cell (Hilbert) order so that the lanes of a
// wave visit the same cells.  The K-1 best candidates live in registers,
// sorted ascending by (d2, id) and right-aligned in an array of KM slots; the
// KM-(K-1) leading slots hold (0, 0), which no candidate can move past, so the
// current worst is always slot KM-1 and every index is a compile-time
// constant.  Cells are searched in Chebyshev shells r = 0, 1, 2, ...; after a
// shell every unvisited vertex is at least `gap` quantisation steps away on
// some axis, so the search stops once the worst kept distance is < gap^2 (a
// candidate at exactly gap could still win on a smaller id).

__device__ inline bool key_less(uint64_t d1, uint32_t o1, uint64_t d2, uint32_t o2) {
    return d1 < d2 || (d1 == d2 && o1 < o2);
}

// Insert (d2, oid) into the sorted, right-aligned list if it beats the worst.
template <int KM>
__device__ __forceinline__ void list_insert(uint64_t (&d)[KM], uint32_t (&o)[KM], uint64_t d2, uint32_t oid) {
    if (key_less(d2, oid, d[KM - 1], o[KM - 1])) {
        d[KM - 1] = d2;
        o[KM - 1] = oid;
#pragma unroll
        for (int p = KM - 1; p > 0; --p) {
            const bool sw = key_less(d[p], o[p], d[p - 1], o[p - 1]);
            const uint64_t td = d[p];
            const uint32_t to = o[p];
            d[p] = sw ? d[p - 1] : d[p];
            o[p] = sw ? o[p - 1] : o[p];
            d[p - 1] = sw ? td : d[p - 1];
            o[p - 1] = sw ? to : o[p - 1];
        }
    }
}

template <int KM>
__device__ __forceinline__ void list_reset(uint64_t (&d)[KM], uint32_t (&o)[KM], int m) {
#pragma unroll
    for (int p = 0; p < KM; ++p) {
        const bool sentinel = p < KM - m;
        d[p] = sentinel ? 0ull : ~0ull;
        o[p] = sentinel ? 0u : ~0u;
    }
}

// Exact search for query s by Chebyshev shells of cells around its own.  A
// cell whose box is farther from q than the current (K-1)-th distance cannot
// contribute and is skipped without reading it (only once the list is full:
// before that the worst key is (inf, inf)); a cell at exactly that distance is
// still read, since a tie may win on id.  Candidates are loaded two at a time.
template <int KM>
__device__ __forceinline__ void shell_search(int64_t s, int m, int shift, int32_t qx, int32_t qy, int32_t qz,
                                             const uint64_t* __restrict__ qs, const int32_t* __restrict__ perm,
                                             const uint2* __restrict__ cell_range, uint64_t (&d)[KM],
                                             uint32_t (&o)[KM]) {
    (void)m;
    const int G = 1 << (kQBits - shift);
    const int cx = qx >> shift, cy = qy >> shift, cz = qz >> shift;
    const int64_t cs = (int64_t)1 << shift;
    for (int r = 0;; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= G) continue;
            const int64_t gz = dz < 0 ? (int64_t)qz - ((int64_t)(z + 1) * cs - 1) : (dz > 0 ? (int64_t)z * cs - qz : 0);
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= G) continue;
                const int64_t gy = dy < 0 ? (int64_t)qy - ((int64_t)(y + 1) * cs - 1) : (dy > 0 ? (int64_t)y * cs - qy : 0);
                const bool face = (dz == -r || dz == r || dy == -r || dy == r);
                const int step = (face || r == 0) ? 1 : 2 * r;
                for (int dx = -r; dx <= r; dx += step) {
                    const int x = cx + dx;
                    if (x < 0 || x >= G) continue;
                    const int64_t gx = dx < 0 ? (int64_t)qx - ((int64_t)(x + 1) * cs - 1) : (dx > 0 ? (int64_t)x * cs - qx : 0);
                    if ((uint64_t)(gx * gx + gy * gy + gz * gz) > d[KM - 1]) continue;   // whole cell too far
                    const uint32_t cell = morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
                    const uint2 cr = cell_range[cell];
                    const uint32_t beg = cr.x, end = cr.y;
                    uint32_t t = beg;
                    for (; t + 1 < end; t += 2) {
                        const uint64_t p0 = qs[t], p1 = qs[t + 1];
                        const uint32_t o0 = (uint32_t)perm[t], o1 = (uint32_t)perm[t + 1];
                        int32_t ax, ay, az;
                        if ((int64_t)t != s) {
                            qunpack(p0, ax, ay, az);
                            const int64_t ex = ax - qx, ey = ay - qy, ez = az - qz;
                            list_insert<KM>(d, o, (uint64_t)(ex * ex + ey * ey + ez * ez), o0);
                        }
                        if ((int64_t)t + 1 != s) {
                            qunpack(p1, ax, ay, az);
                            const int64_t ex = ax - qx, ey = ay - qy, ez = az - qz;
                            list_insert<KM>(d, o, (uint64_t)(ex * ex + ey * ey + ez * ez), o1);
                        }
                    }
                    if (t < end && (int64_t)t != s) {
                        int32_t ax, ay, az;
                        qunpack(qs[t], ax, ay, az);
                        const int64_t ex = ax - qx, ey = ay - qy, ez = az - qz;
                        list_insert<KM>(d, o, (uint64_t)(ex * ex + ey * ey + ez * ez), (uint32_t)perm[t]);
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
            if (c3[a] - r > 0) gap = min(gap, q3[a] - (int64_t)(c3[a] - r) * cs + 1);
            if (c3[a] + r < G - 1) gap = min(gap, (int64_t)(c3[a] + r + 1) * cs - q3[a]);
        }
        if (gap == INT64_MAX) break;                    // the whole grid was searched
        if (d[KM - 1] < (uint64_t)(gap * gap)) break;   // list full and provably final
    }
}

template <int KM>
__device__ __forceinline__ void knn_write(int64_t s, int K, int m, uint32_t self, int64_t N, const int32_t* inv,
                                          const uint64_t (&d)[KM], const uint32_t (&o)[KM], int32_t* col_sorted,
                                          int32_t* col_canon, int64_t* row_ptr) {
    (void)d;
    if (col_sorted) {   // sliced-ELL layout; the padding slots of the row's last quad point at itself
        col_sorted[eidx(s, 0, K)] = (int32_t)s;
#pragma unroll
        for (int p = 0; p < KM; ++p)
            if (p >= KM - m) col_sorted[eidx(s, 1 + p - (KM - m), K)] = inv[o[p]];
        for (int l = K; l < ell_k4(K); ++l) col_sorted[eidx(s, l, K)] = (int32_t)s;
    }
    if (col_canon) {
        int32_t* row = col_canon + (int64_t)self * K;
        row[0] = (int32_t)self;
#pragma unroll
        for (int p = 0; p < KM; ++p)
            if (p >= KM - m) row[1 + p - (KM - m)] = (int32_t)o[p];
    }
    if (row_ptr) {
        row_ptr[self] = (int64_t)self * K;
        if (s == 0) row_ptr[N] = N * (int64_t)K;
    }
}

// ---- fast path: one 64-bit key per candidate --------------------------
// key = (min(d2, sat) << idb) | id, with idb = the bits ids of this scene need
// (N - 1 < 2^idb) and sat = 2^(64 - idb) - 1, orders exactly like (d2, id) as
// long as d2 < sat.  Every scene below 2^25 vertices keeps 39 distance bits
// (no saturation below ~70% of the unit cube); at 2^31 vertices 33 bits
// (~8.8%).  A k-th neighbour that far saturates the key, and that query is
// redone by the exact search.
struct KeyFmt {
    int idb;
    uint64_t sat, idmask;
};

inline KeyFmt key_fmt(int64_t N) {
    int idb = 1;
    while (idb < 31 && ((int64_t)1 << idb) < N) ++idb;
    return KeyFmt{idb, (~0ull) >> idb, ((uint64_t)1 << idb) - 1};
}

__device__ __forceinline__ uint64_t make_key(uint64_t d2, uint32_t oid, const KeyFmt& f) {
    return ((d2 < f.sat ? d2 : f.sat) << f.idb) | (uint64_t)oid;
}

// Insert c into the ascending list if it beats the last key, as a merge: slot
// p keeps its key if c is not below it, takes c if c falls between slots p-1
// and p, and the key of slot p-1 otherwise.  The comparisons against c are
// independent of each other (a bubble pass would chain them), and each slot
// costs one 64-bit compare and two selects.
template <int KM>
__device__ __forceinline__ void key_insert(uint64_t (&k)[KM], uint64_t c) {
    if (c < k[KM - 1]) {
        bool lt[KM];
        uint64_t v[KM];
#pragma unroll
        for (int p = 0; p < KM; ++p) {
            lt[p] = c < k[p];
            // an empty asm hides that v[p] equals k[p]: the selects below then
            // reuse lt[] instead of being rebuilt as min/max with compares of their own
            v[p] = k[p];
            asm("" : "+v"(v[p]));
        }
#pragma unroll
        for (int p = KM - 1; p > 0; --p) k[p] = lt[p] ? (lt[p - 1] ? v[p - 1] : c) : v[p];
        k[0] = lt[0] ? c : v[0];
    }
}

// The list is seeded with the kKnnWin vertices on either side of the query in
// cell order (the same trip count on every lane, loads coalesced across the
// wave), which gives the shells a tight bound to prune cells with from the
// start; the shells then skip that index range, so every vertex is offered
// once.  Seeding with 16 on either side: kNN 5% faster on the 68.8M-vertex
// cloud at the finest cell size, unchanged on the 22M-vertex ball.
constexpr int kKnnWin = 16;

template <int KM>
__device__ __forceinline__ void key_shell_search(int64_t N, int64_t s, int shift, int32_t qx, int32_t qy, int32_t qz,
                                                 const uint64_t* __restrict__ qs, const int32_t* __restrict__ perm,
                                                 const uint2* __restrict__ cell_range, const KeyFmt f,
                                                 uint64_t (&k)[KM]) {
    const int64_t lo = s - kKnnWin < 0 ? 0 : s - kKnnWin;
    const int64_t hi = s + kKnnWin >= N ? N - 1 : s + kKnnWin;
    for (int o = -kKnnWin; o <= kKnnWin; ++o) {
        const int64_t t = s + o;
        if (o == 0 || t < 0 || t >= N) continue;
        int32_t ax, ay, az;
        qunpack(qs[t], ax, ay, az);
        const int64_t ex = ax - qx, ey = ay - qy, ez = az - qz;
        key_insert<KM>(k, make_key((uint64_t)(ex * ex + ey * ey + ez * ez), (uint32_t)perm[t], f));
    }
    const int G = 1 << (kQBits - shift);
    const int cx = qx >> shift, cy = qy >> shift, cz = qz >> shift;
    const int64_t cs = (int64_t)1 << shift;
    for (int r = 0;; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= G) continue;
            const int64_t gz = dz < 0 ? (int64_t)qz - ((int64_t)(z + 1) * cs - 1) : (dz > 0 ? (int64_t)z * cs - qz : 0);
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= G) continue;
                const int64_t gy = dy < 0 ? (int64_t)qy - ((int64_t)(y + 1) * cs - 1) : (dy > 0 ? (int64_t)y * cs - qy : 0);
                const bool face = (dz == -r || dz == r || dy == -r || dy == r);
                const int step = (face || r == 0) ? 1 : 2 * r;
                for (int dx = -r; dx <= r; dx += step) {
                    const int x = cx + dx;
                    if (x < 0 || x >= G) continue;
                    const int64_t gx = dx < 0 ? (int64_t)qx - ((int64_t)(x + 1) * cs - 1) : (dx > 0 ? (int64_t)x * cs - qx : 0);
                    if ((uint64_t)(gx * gx + gy * gy + gz * gz) > (k[KM - 1] >> f.idb)) continue;   // cell too far
                    const uint32_t cell = morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
                    const uint2 cr = cell_range[cell];
                    const uint32_t beg = cr.x, end = cr.y;
                    for (uint32_t t = beg; t < end; ++t) {
                        if ((int64_t)t >= lo && (int64_t)t <= hi) continue;   // seeded (or the query)
                        int32_t ax, ay, az;
                        qunpack(qs[t], ax, ay, az);
                        const int64_t ex = ax - qx, ey = ay - qy, ez = az - qz;
                        key_insert<KM>(k, make_key((uint64_t)(ex * ex + ey * ey + ez * ez), (uint32_t)perm[t], f));
                    }
                }
            }
        }
        int64_t gap = INT64_MAX;
        const int c3[3] = {cx, cy, cz};
        const int64_t q3[3] = {qx, qy, qz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c3[a] - r > 0) gap = min(gap, q3[a] - (int64_t)(c3[a] - r) * cs + 1);
            if (c3[a] + r < G - 1) gap = min(gap, (int64_t)(c3[a] + r + 1) * cs - q3[a]);
        }
        if (gap == INT64_MAX) break;
        if ((k[KM - 1] >> f.idb) < (uint64_t)(gap * gap)) break;
    }
}

// WPE: the minimum waves per SIMD the compiler must fit the search in.  For
// lists of up to 16 keys a bound of 6 or 8 (whichever compiles without
// spills: 8 for 7 and 9-14 keys, 6 for 8, 15 and 16) fits it in 55-68
// registers, 7-8 resident waves instead of 4, which hides more of the
// candidate loads' latency (at 15 keys the bound of 6 ran 3% faster than 8);
// longer lists take no bound (1).
template <int KM, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_knn(int64_t N, int K, int shift, const uint64_t* __restrict__ qs,
                                                const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                                                const uint2* __restrict__ cell_range,
                                                int32_t* __restrict__ col_sorted, int32_t* __restrict__ col_canon,
                                                int64_t* __restrict__ row_ptr, uint32_t* __restrict__ redo,
                                                uint32_t* __restrict__ nredo, const KeyFmt f) {
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t s = tile * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int m = K - 1;
    int32_t qx, qy, qz;
    qunpack(qs[s], qx, qy, qz);
    const uint32_t self = (uint32_t)perm[s];
    uint64_t k[KM];
#pragma unroll
    for (int p = 0; p < KM; ++p) k[p] = p < KM - m ? 0ull : ~0ull;
    if (m > 0) key_shell_search<KM>(N, s, shift, qx, qy, qz, qs, perm, cell_range, f, k);
    const bool sat = m > 0 && (k[KM - 1] >> f.idb) >= f.sat;   // a kept distance saturated: redo exactly
    const uint32_t slot = wave_append(nredo, sat);
    if (sat) {
        redo[slot] = (uint32_t)s;
        return;
    }
    if (col_sorted) {   // sliced-ELL layout; the padding slots of the row's last quad point at itself
        col_sorted[eidx(s, 0, K)] = (int32_t)s;
#pragma unroll
        for (int p = 0; p < KM; ++p)
            if (p >= KM - m) col_sorted[eidx(s, 1 + p - (KM - m), K)] = inv[(uint32_t)(k[p] & f.idmask)];
        for (int l = K; l < ell_k4(K); ++l) col_sorted[eidx(s, l, K)] = (int32_t)s;
    }
    if (col_canon) {
        int32_t* row = col_canon + (int64_t)self * K;
        row[0] = (int32_t)self;
#pragma unroll
        for (int p = 0; p < KM; ++p)
            if (p >= KM - m) row[1 + p - (KM - m)] = (int32_t)(k[p] & f.idmask);
    }
    if (row_ptr) {
        row_ptr[self] = (int64_t)self * K;
        if (s == 0) row_ptr[N] = N * (int64_t)K;
    }
}

// Exact (d2, id) search for the queries the fast path handed over.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_knn_exact(int64_t N, int K, int shift, const uint64_t* __restrict__ qs,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ inv,
                                                      const uint2* __restrict__ cell_range,
                                                      int32_t* __restrict__ col_sorted,
                                                      int32_t* __restrict__ col_canon,
                                                      int64_t* __restrict__ row_ptr,
                                                      const uint32_t* __restrict__ redo,
                                                      const uint32_t* __restrict__ nredo) {
    const uint32_t n = *nredo;
    const int m = K - 1;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
        const int64_t s = redo[idx];
        int32_t qx, qy, qz;
        qunpack(qs[s], qx, qy, qz);
        const uint32_t self = (uint32_t)perm[s];
        uint64_t d[KM];
        uint32_t o[KM];
        list_reset<KM>(d, o, m);
        shell_search<KM>(s, m, shift, qx, qy, qz, qs, perm, cell_range, d, o);
        knn_write<KM>(s, K, m, self, N, inv, d, o, col_sorted, col_canon, row_ptr);
    }
}

// Every query handed to the exact search (PG_FLAG_EXACT_KNN).
__global__ __launch_bounds__(kBlock) void k_redo_all(int64_t N, uint32_t* __restrict__ redo,
                                                     uint32_t* __restrict__ nredo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) redo[i] = (uint32_t)i;
    if (i == 0) *nredo = (uint32_t)N;
}

hipError_t launch_knn(int64_t N, int K, int shift, const uint64_t* qsorted, const int32_t* perm,
                      const int32_t* inv, const uint2* cell_range, int32_t* col_sorted, int32_t* col_canon,
                      int64_t* row_ptr, uint32_t* redo, uint32_t* nredo, bool exact_only, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int m = K - 1;
    hipError_t e = launch_fill(nredo, sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    const KeyFmt f = key_fmt(N);
    auto go = [&](auto km) {
        constexpr int KM = decltype(km)::value;
        constexpr int WPE = KM == 8 ? 6 : (KM <= 14 ? 8 : (KM <= 16 ? 6 : 1));
        if (exact_only)
            hipLaunchKernelGGL(k_redo_all, dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, redo, nredo);
        else
            hipLaunchKernelGGL((k_knn<KM, WPE>), dim3((unsigned)div_up(N, kBlock)), dim3(kBlock), 0, s, N, K,
                               shift, qsorted, perm, inv, cell_range, col_sorted, col_canon, row_ptr, redo, nredo,
                               f);
        hipLaunchKernelGGL(k_knn_exact<KM>, dim3(256), dim3(kBlock), 0, s, N, K, shift, qsorted, perm, inv,
                           cell_range, col_sorted, col_canon, row_ptr, (const uint32_t*)redo,
                           (const uint32_t*)nredo);
    };
    // k = 8..17 get a list of exactly K-1 keys: a sentinel slot costs its
    // compare and selects in every insertion
    switch (m) {
        case 7: go(std::integral_constant<int, 7>{}); break;
        case 8: go(std::integral_constant<int, 8>{}); break;
        case 9: go(std::integral_constant<int, 9>{}); break;
        case 10: go(std::integral_constant<int, 10>{}); break;
        case 11: go(std::integral_constant<int, 11>{}); break;
        case 12: go(std::integral_constant<int, 12>{}); break;
        case 13: go(std::integral_constant<int, 13>{}); break;
        case 14: go(std::integral_constant<int, 14>{}); break;
        case 15: go(std::integral_constant<int, 15>{}); break;
        case 16: go(std::integral_constant<int, 16>{}); break;
        default:
            if (m < 7) go(std::integral_constant<int, 8>{});
            else if (m <= 32) go(std::integral_constant<int, 32>{});
            else go(std::integral_constant<int, 64>{});
    }
    return hipGetLastError();
}

}  // namespace pg
