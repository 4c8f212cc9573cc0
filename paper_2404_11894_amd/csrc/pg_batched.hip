// pg_batched.hip -- many independent scenes per launch.
//
// Each scene gets its own slice of the workspace (the same buffers as a
// single render).  A scene with the cluster relation runs its setup and its
// own iterations on its setup stream, beside the batched loop of the others.  The one-time steps (grid, kNN, weights, path pass, pixels)
// run per scene, spread over a few streams; the D iterations -- the hot loop
// -- run as ONE spmv launch and ONE shift launch for all scenes per
// iteration: a block finds its scene in a small descriptor table and leaves
// at once when its scene has finished its own D iterations.
// A pg_batch plan can capture the whole sequence in a hipGraph, so a render
// of all scenes is one graph launch.
#include <algorithm>
#include <vector>

#include "pg_api_common.h"

namespace pg {

struct SceneDesc {
    const int32_t* col;
    const int16_t* c16;          // compact ids (NULL: the 32-bit ids)
    const uint32_t* c16_base;
    const int32_t* c16_ovf;
    const float* w;
    const float* b;
    const float* alpha;
    const int32_t* succ;
    float* x;
    float* y;
    int64_t nrows;
    int64_t blk0;     // first block of this scene in the batched launch
    int32_t K, D;
};

// Blocks of the scenes still iterating at step t: the tables are ordered by
// decreasing D, so those scenes are a prefix.
__host__ __device__ inline int64_t active_blocks(const SceneDesc* sd, int n, int t, int64_t nblk) {
    int lo = 0, hi = n;   // first entry with D < t
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sd[mid].D >= t) lo = mid + 1;
        else hi = mid;
    }
    return lo < n ? sd[lo].blk0 : nblk;
}

__device__ inline int find_scene(const SceneDesc* sd, int n, int64_t blk) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sd[mid].blk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// y_i = b_i + alpha_i sum_l w_il x(j_l) for every row of every scene still
// iterating (t <= D_s); one thread per row over each scene's sliced-ELL
// edges.  A block belongs to one scene, so the branch on the scene's K4 is
// uniform: K4 = 8, 12, 16 take the unrolled row sum, other counts the loop.
template <int KT>
__device__ __forceinline__ void spmv_batched_row(const SceneDesc& d, int64_t i) {
    f3 z;
    if constexpr (KT > 0) {
        if (d.c16) z = c16_row_sum<KT>(i, d.K, d.c16, d.c16_base, d.c16_ovf, d.w, d.x);
        else z = ell_row_sum<KT>(i, d.K, d.col, d.w, d.x);
    } else {
        z = ell_row_sum<KT>(i, d.K, d.col, d.w, d.x);
    }
    const float a = d.alpha[i];
    const f3 bb = ld3(d.b, i);
    st3_nt(d.y, i, f3{fmaf(a, z.x, bb.x), fmaf(a, z.y, bb.y), fmaf(a, z.z, bb.z)});
}

// Workgroups of BS rows; tile_group as in the single-scene aggregation.
template <int BS>
__global__ __launch_bounds__(BS) void k_spmv_batched(const SceneDesc* __restrict__ sd, int nsc, int t, int group) {
    const int64_t blk = grouped_tile(blockIdx.x, gridDim.x, group);
    const SceneDesc& d = sd[find_scene(sd, nsc, blk)];
    if (t > d.D) return;
    const int64_t i = (blk - d.blk0) * (int64_t)BS + threadIdx.x;
    if (i >= d.nrows) return;
    switch (ell_k4(d.K)) {
    case 8: spmv_batched_row<8>(d, i); break;
    case 12: spmv_batched_row<12>(d, i); break;
    case 16: spmv_batched_row<16>(d, i); break;
    default: spmv_batched_row<0>(d, i); break;
    }
}

// x(v) = y(succ v), 0 at a path's end, for scenes still iterating.
template <int BS>
__global__ __launch_bounds__(BS) void k_shift_batched(const SceneDesc* __restrict__ sd, int nsc, int t) {
    const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);   // as the single-scene shift
    const SceneDesc& d = sd[find_scene(sd, nsc, blk)];
    if (t > d.D) return;
    const int64_t v = (blk - d.blk0) * (int64_t)blockDim.x + threadIdx.x;
    if (v >= d.nrows) return;
    const int64_t u = __builtin_nontemporal_load(d.succ + v);
    f3 val{0.f, 0.f, 0.f};
    if (u >= 0) val = ld3(d.y, u);
    st3_nt(d.x, v, val);
}

// ----------------------------------------- persistent schedule (opt-in) ---
// PG_FLAG_PERSISTENT: one cooperative launch runs every iteration of every
// scene, a grid-stride loop over the same virtual blocks as the per-iteration
// launches, with a grid barrier between the aggregation and the shift and
// between iterations.  The cooperative launch makes every workgroup resident
// at once, so every barrier is reached; the wait is still bounded (spin_limit
// sleeps, about a second): a workgroup that runs out sets the abort word and
// every workgroup leaves at its next barrier, and the host reports it.  Each
// barrier is a device-scope release and acquire by every workgroup (the XCDs'
// L2 caches are not coherent with each other), which costs more than the
// kernel boundaries of the default schedule.
__device__ bool grid_barrier(uint32_t* count, uint32_t* abortf, uint32_t target, uint32_t spin_limit) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        __threadfence();
        atomicAdd(count, 1u);
        uint32_t n = 0;
        while (__hip_atomic_load(count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++n > spin_limit) {
                atomicOr(abortf, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __threadfence();
    }
    __syncthreads();
    return ok != 0;
}

__global__ __launch_bounds__(kBlock) void k_batch_persistent(const SceneDesc* __restrict__ sd, int nsc, int Dmax,
                                                             int64_t nblk, uint32_t* bar, uint32_t spin_limit) {
    uint32_t phase = 0;
    for (int t = 1; t <= Dmax; ++t) {
        const int64_t nb = active_blocks(sd, nsc, t, nblk);
        for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
            const SceneDesc& d = sd[find_scene(sd, nsc, b)];
            if (t > d.D) continue;
            const int64_t i = (b - d.blk0) * (int64_t)kBlock + threadIdx.x;
            if (i >= d.nrows) continue;
            switch (ell_k4(d.K)) {
            case 8: spmv_batched_row<8>(d, i); break;
            case 12: spmv_batched_row<12>(d, i); break;
            case 16: spmv_batched_row<16>(d, i); break;
            default: spmv_batched_row<0>(d, i); break;
            }
        }
        if (!grid_barrier(bar, bar + 1, ++phase * gridDim.x, spin_limit)) return;
        for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
            const SceneDesc& d = sd[find_scene(sd, nsc, b)];
            if (t > d.D) continue;
            const int64_t v = (b - d.blk0) * (int64_t)kBlock + threadIdx.x;
            if (v >= d.nrows) continue;
            const int64_t u = __builtin_nontemporal_load(d.succ + v);
            f3 val{0.f, 0.f, 0.f};
            if (u >= 0) val = ld3(d.y, u);
            st3_nt(d.x, v, val);
        }
        if (!grid_barrier(bar, bar + 1, ++phase * gridDim.x, spin_limit)) return;
    }
}

// ------------------------------------------------------------------ host ---

struct BatchLayout {
    int n = 0;
    std::vector<RenderBufs> r;
    std::vector<pg_params> q;
    // one descriptor per scene with vertices; `tile` rows per block (the first
    // scene's params->tile, 0 = 256), tile_group likewise
    int tile = kBlock, tile_group = 1;
    int64_t blocks = 0;
    std::vector<SceneDesc> host_tables;
    SceneDesc* dev_tables = nullptr;
    uint32_t* bar = nullptr;   // persistent schedule: barrier counter, abort word
    bool persistent = false;
    int Dmax = 0;
};

// Carves every scene's buffers and the descriptor tables; with a real base
// also fills the host copy of the tables.
static void carve_batch(Carver& cv, BatchLayout& L, int n, const pg_paths* paths, const pg_params* params) {
    L.n = n;
    L.r.assign(n, RenderBufs());
    L.q.assign(params, params + n);
    for (int s = 0; s < n; ++s) {
        L.q[s].schedule = PG_SCHED_TWO_PASS;
        L.q[s].flags &= ~PG_FLAG_TAPE;
        carve_render(cv, L.r[s], &paths[s], &L.q[s]);
    }
    L.host_tables.clear();
    L.Dmax = 0;
    L.tile = params[0].tile ? params[0].tile : kBlock;
    L.persistent = (params[0].flags & PG_FLAG_PERSISTENT) != 0;
    L.tile_group = params[0].tile_group ? params[0].tile_group : 1;
    // tables in decreasing order of D (ties by scene), so that the scenes
    // still iterating at any step own a prefix of the blocks
    std::vector<int> order;
    for (int s = 0; s < n; ++s)
        if (L.r[s].N > 0 && !L.r[s].clusters) order.push_back(s);   // cluster scenes iterate on their own stream
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L.r[a].D > L.r[b].D; });
    int64_t blk = 0;
    for (int s : order) {
        const RenderBufs& r = L.r[s];
        if (r.D > L.Dmax) L.Dmax = r.D;
        SceneDesc d{r.col, r.c16, r.c16_base, r.c16_ovf, r.w, r.b, r.alpha, r.succ, r.x, r.y, r.N, blk, r.K, r.D};
        L.host_tables.push_back(d);
        blk += div_up(r.N, L.tile);
    }
    L.blocks = blk;
    L.dev_tables = cv.take<SceneDesc>((int64_t)(L.host_tables.size() > 0 ? L.host_tables.size() : 1));
    L.bar = cv.take<uint32_t>(64);
}

static pg_status validate_batch(int n, const pg_paths* paths, const pg_params* params) {
    if (n < 1) return fail(PG_ERR_ARG, "n_scenes must be >= 1");
    if (!paths || !params) return fail(PG_ERR_ARG, "paths and params are required");
    for (int s = 0; s < n; ++s) {
        pg_status st;
        if ((st = validate_paths(&paths[s], true)) || (st = validate_params(&params[s])))
            return fail(st, "scene %d: %s", s, g_error.c_str());
        pg_params qs = params[s];
        qs.schedule = PG_SCHED_TWO_PASS;
        qs.flags &= ~PG_FLAG_TAPE;
        if ((st = validate_clusters(&paths[s], &qs))) return fail(st, "scene %d: %s", s, g_error.c_str());
    }
    if ((params[0].flags & PG_FLAG_PERSISTENT) && params[0].tile != 0 && params[0].tile != kBlock)
        return fail(PG_ERR_UNSUPPORTED, "PG_FLAG_PERSISTENT runs workgroups of 256 rows (tile 0 or 256)");
    return PG_OK;
}

// Phase B: the D iterations of every scene, batched.
static hipError_t batched_iterations(const BatchLayout& L, hipStream_t s) {
    const int nsc = (int)L.host_tables.size();
    if (L.persistent && L.blocks > 0 && L.Dmax > 0) {
        int dev = 0, ncu = 0, per_cu = 0;
        hipError_t e;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, kBlock, 0)) != hipSuccess)
            return e;
        int64_t grid = (int64_t)ncu * per_cu;
        if (grid > L.blocks) grid = L.blocks;
        if (grid < 1) grid = 1;
        if ((e = launch_fill(L.bar, 64 * 4, s)) != hipSuccess) return e;
        const SceneDesc* sdp = L.dev_tables;
        int nscv = nsc, dmax = L.Dmax;
        int64_t nblk = L.blocks;
        uint32_t* bar = L.bar;
        uint32_t spin = 1u << 22;
        void* args[] = {(void*)&sdp, (void*)&nscv, (void*)&dmax, (void*)&nblk, (void*)&bar, (void*)&spin};
        ProfScope ps(s, "batched_persistent");
        return hipLaunchCooperativeKernel((const void*)k_batch_persistent, dim3((unsigned)grid), dim3(kBlock), args,
                                          0, s);
    }
    if (L.persistent) return hipSuccess;   // nothing to iterate
    for (int t = 1; t <= L.Dmax && L.blocks > 0; ++t) {
        const int64_t nb = active_blocks(L.host_tables.data(), nsc, t, L.blocks);   // scenes with D >= t
        dispatch_tile(L.tile, [&](auto bs) {
            constexpr int BS = decltype(bs)::value;
            {
                ProfScope ps(s, "spmv_batched");
                hipLaunchKernelGGL(k_spmv_batched<BS>, dim3((unsigned)nb), dim3(BS), 0, s, L.dev_tables, nsc, t,
                                   L.tile_group);
            }
            ProfScope ps(s, "shift_batched");
            hipLaunchKernelGGL(k_shift_batched<BS>, dim3((unsigned)nb), dim3(BS), 0, s, L.dev_tables, nsc, t);
        });
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Stream of each scene's setup and output: largest first (by N K, the cost
// of its kNN and weights) onto the least-loaded of the ns streams.
static std::vector<int> stream_of_scene(const BatchLayout& L, int ns) {
    std::vector<int> order(L.n), which(L.n, 0);
    for (int s = 0; s < L.n; ++s) order[s] = s;
    auto cost = [&](int s) { return (double)L.r[s].N * (double)(L.r[s].K > 0 ? L.r[s].K : 1); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<double> load(ns, 0.0);
    for (int s : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        which[s] = k;
        load[k] += cost(s);
    }
    return which;
}

// Runs all three phases.  Streams: the setup and output of each scene go to
// the stream stream_of_scene picks; streams[0] is the caller's and does the
// batched loop.
static hipError_t run_batch(const pg_paths* paths, BatchLayout& L, float* const* images, hipStream_t* streams,
                            int ns, hipEvent_t* ev) {
    hipStream_t s0 = streams[0];
    hipError_t e;
    const std::vector<int> which = stream_of_scene(L, ns);
    if (ns > 1) {
        if ((e = hipEventRecord(ev[0], s0)) != hipSuccess) return e;
        for (int k = 1; k < ns; ++k)
            if ((e = hipStreamWaitEvent(streams[k], ev[0], 0)) != hipSuccess) return e;
    }
    for (int s = 0; s < L.n; ++s) {
        float* x0 = nullptr;
        if (L.r[s].clusters) {   // the cluster relation: setup and its own iterations on the scene's stream
            float* xD = nullptr;
            if ((e = cluster_setup(&paths[s], &L.q[s], L.r[s], nullptr, streams[which[s]], &x0)) != hipSuccess)
                return e;
            if ((e = cluster_iterate(L.r[s], &L.q[s], x0, streams[which[s]], &xD)) != hipSuccess) return e;
            continue;
        }
        if ((e = render_setup(&paths[s], &L.q[s], L.r[s], nullptr, streams[which[s]], &x0)) != hipSuccess)
            return e;
    }
    if (ns > 1) {
        for (int k = 1; k < ns; ++k) {
            if ((e = hipEventRecord(ev[k], streams[k])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s0, ev[k], 0)) != hipSuccess) return e;
        }
    }
    if ((e = batched_iterations(L, s0)) != hipSuccess) return e;
    if (ns > 1) {
        if ((e = hipEventRecord(ev[0], s0)) != hipSuccess) return e;
        for (int k = 1; k < ns; ++k)
            if ((e = hipStreamWaitEvent(streams[k], ev[0], 0)) != hipSuccess) return e;
    }
    for (int s = 0; s < L.n; ++s) {
        e = L.r[s].clusters ? cluster_output(&paths[s], &L.q[s], L.r[s], nullptr, images[s], L.r[s].x, streams[which[s]])
                            : render_output(&paths[s], &L.q[s], L.r[s], nullptr, images[s], L.r[s].x, streams[which[s]]);
        if (e != hipSuccess) return e;
    }
    if (ns > 1) {
        for (int k = 1; k < ns; ++k) {
            if ((e = hipEventRecord(ev[k], streams[k])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s0, ev[k], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

static size_t batch_size(int n, const pg_paths* paths, const pg_params* params) {
    Carver cv(nullptr);
    BatchLayout L;
    carve_batch(cv, L, n, paths, params);
    return cv.size();
}

}  // namespace pg

using namespace pg;

struct pg_batch {
    int n = 0;
    std::vector<pg_paths> paths;
    std::vector<float*> images;
    BatchLayout L;
    int ns = 1;
    hipStream_t streams[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool own_streams = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t flags = 0;
};

static void destroy_batch(pg_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int k = 0; k < 4; ++k) {
        if (b->ev[k]) (void)hipEventDestroy(b->ev[k]);
        if (b->own_streams && k > 0 && b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
    }
    delete b;
}

extern "C" {

pg_status pg_render_batched_workspace_size(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                                           size_t* bytes) {
    g_error.clear();
    pg_status st = validate_batch(n_scenes, paths, params);
    if (st) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    *bytes = batch_size(n_scenes, paths, params);
    return PG_OK;
}

pg_status pg_batch_create(int32_t n_scenes, const pg_paths* paths, const pg_params* params, float* const* images,
                          void* ws, size_t ws_bytes, int32_t use_graph, void* stream, pg_batch** out) {
    g_error.clear();
    pg_status st = validate_batch(n_scenes, paths, params);
    if (st) return st;
    if (!images || !out) return fail(PG_ERR_ARG, "images and out are required");
    if (use_graph && !stream) return fail(PG_ERR_ARG, "graph capture needs a created stream, not the null stream");
    for (int s = 0; s < n_scenes; ++s)
        if (!images[s]) return fail(PG_ERR_ARG, "images[%d] is NULL", s);
    if ((st = check_ws(ws, ws_bytes, batch_size(n_scenes, paths, params)))) return st;
    pg_batch* b = new (std::nothrow) pg_batch();
    if (!b) return fail(PG_ERR_ARG, "out of host memory");
    b->n = n_scenes;
    b->paths.assign(paths, paths + n_scenes);
    b->images.assign(images, images + n_scenes);
    Carver cv(ws);
    carve_batch(cv, b->L, n_scenes, b->paths.data(), params);
    for (int s = 0; s < n_scenes; ++s) b->L.q[s].flags &= ~PG_FLAG_CHECK;
    hipStream_t s0 = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    // the descriptor tables go to the device once, before any capture
    if (!b->L.host_tables.empty()) {
        e = hipMemcpyAsync(b->L.dev_tables, b->L.host_tables.data(), b->L.host_tables.size() * sizeof(SceneDesc),
                           hipMemcpyHostToDevice, s0);
        if (e == hipSuccess) e = hipStreamSynchronize(s0);
    }
    b->ns = n_scenes > 1 ? 4 : 1;
    b->streams[0] = s0;
    b->own_streams = true;
    for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming);
    for (int k = 1; k < b->ns && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_batch(b);
        return hip_fail(e, "pg_batch_create");
    }
    if (use_graph) {
        e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t er = run_batch(b->paths.data(), b->L, b->images.data(), b->streams, b->ns, b->ev);
            e = hipStreamEndCapture(s0, &b->graph);
            if (er != hipSuccess) e = er;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            destroy_batch(b);
            return hip_fail(e, "graph capture");
        }
    }
    *out = b;
    return PG_OK;
}

pg_status pg_batch_launch(pg_batch* b, void* stream) {
    g_error.clear();
    if (!b) return fail(PG_ERR_ARG, "batch is NULL");
    hipStream_t s0 = (hipStream_t)stream;
    hipError_t e;
    if (b->exec) {
        e = hipGraphLaunch(b->exec, s0);
    } else {
        hipStream_t st[4] = {s0, b->streams[1], b->streams[2], b->streams[3]};
        e = run_batch(b->paths.data(), b->L, b->images.data(), st, b->ns, b->ev);
    }
    if (e != hipSuccess) return hip_fail(e, "pg_batch_launch");
    return PG_OK;
}

pg_status pg_batch_destroy(pg_batch* b) {
    g_error.clear();
    destroy_batch(b);
    return PG_OK;
}

pg_status pg_render_batched(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                            float* const* images, void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st = validate_batch(n_scenes, paths, params);
    if (st) return st;
    if (!images) return fail(PG_ERR_ARG, "images is NULL");
    for (int s = 0; s < n_scenes; ++s)
        if (!images[s]) return fail(PG_ERR_ARG, "images[%d] is NULL", s);
    if ((st = check_ws(ws, ws_bytes, batch_size(n_scenes, paths, params)))) return st;
    Carver cv(ws);
    BatchLayout L;
    carve_batch(cv, L, n_scenes, paths, params);
    hipStream_t s0 = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!L.host_tables.empty()) {
        e = hipMemcpyAsync(L.dev_tables, L.host_tables.data(), L.host_tables.size() * sizeof(SceneDesc),
                           hipMemcpyHostToDevice, s0);
        // the host copy of the tables dies with this call
        if (e == hipSuccess) e = hipStreamSynchronize(s0);
    }
    hipStream_t one[1] = {s0};
    if (e == hipSuccess) e = run_batch(paths, L, images, one, 1, nullptr);
    if (e != hipSuccess) return hip_fail(e, "pg_render_batched");
    if (L.persistent && L.blocks > 0 && L.Dmax > 0) {   // the persistent schedule's abort word
        uint32_t ab = 0;
        if ((e = hipMemcpyAsync(&ab, L.bar + 1, sizeof ab, hipMemcpyDeviceToHost, s0)) != hipSuccess ||
            (e = hipStreamSynchronize(s0)) != hipSuccess)
            return hip_fail(e, "pg_render_batched");
        if (ab) return fail(PG_ERR_HIP, "PG_FLAG_PERSISTENT: a grid barrier timed out; the images are not valid");
    }
    uint32_t fl = 0;
    for (int s = 0; s < n_scenes; ++s) fl |= params[s].flags;
    if (fl & (PG_FLAG_CHECK | PG_FLAG_CLUSTERS)) {   // the cluster relation always reports its checks
        for (int s = 0; s < n_scenes; ++s) {
            pg_status fs = finish(s0, &params[s], L.r[s].g.flag, PG_FLAG_CHECK);
            if (fs) return fail(fs, "scene %d: %s", s, g_error.c_str());
        }
    }
    return PG_OK;
}

}  // extern "C"
