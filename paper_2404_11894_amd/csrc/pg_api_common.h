// pg_api_common.h -- host-side helpers shared by the entry points: error
// reporting, workspace carving and the render pipeline used by pg_render,
// pg_backward and pg_render_batched.
#pragma once

#include <string>

#include "pg_internal.h"

namespace pg {

// Sum of one double per thread over the block; the result is valid in thread 0.
__device__ inline double block_sum_d(double v) {
    __shared__ double sh[kBlock / kWave];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / kWave; ++w) t += sh[w];
    return t;
}

__device__ inline float dot3(f3 a, f3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

extern thread_local std::string g_error;
pg_status fail(pg_status code, const char* fmt, ...);
pg_status hip_fail(hipError_t e, const char* where);
pg_status validate_paths(const pg_paths* p, bool need_records);
pg_status validate_params(const pg_params* q);
pg_status validate_clusters(const pg_paths* p, const pg_params* q);
pg_status check_ws(void* ws, size_t ws_bytes, size_t need);
pg_status finish(hipStream_t s, const pg_params* q, const int32_t* dflag, uint32_t flags);
pg_status no_clusters(const pg_params* q);
pg_status check_knn_layout(const pg_params* q, int64_t N, int K, const int64_t* row_ptr, int32_t* flag,
                           hipStream_t s);
Consts make_consts(const pg_params* q, int K);
int32_t default_shift(int64_t N);
int shift_of(const pg_params* q, int64_t N);
// pg_propagate after g_error is cleared: validation, the workspace check
// against propagate_size, and the launches (shared with pg_propagate_static).
size_t propagate_size(const pg_paths* p, const pg_params* q);
pg_status propagate_run(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                        const float* w_ind, const float* b, float* lplus, float* traj, void* ws, size_t ws_bytes,
                        hipStream_t s);

// Brackets one kernel step with HIP events on its stream while profiling is on.
struct ProfScope {
    int slot = -1;
    hipStream_t s;
    ProfScope(hipStream_t stream, const char* name);
    ~ProfScope();
};

// Sub-allocates a workspace in 256-byte aligned pieces.  With a NULL base it
// only measures.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (size_t)(count > 0 ? count : 0) * sizeof(T);
        return p;
    }
    size_t size() const { return (off + 255) & ~(size_t)255; }
};

struct GridBufs {
    int shift = 0;
    int64_t ncells = 0;
    int32_t* flag = nullptr;
    uint32_t* cells = nullptr;     // counts, then start by Hilbert position (ncells + 1)
    uint2* range = nullptr;        // [start, end) of each cell by Morton number (ncells)
    uint32_t* partials = nullptr;
    uint32_t* cellid = nullptr;
    uint32_t* rank = nullptr;
    int32_t* perm = nullptr;       // sorted -> path order
    int32_t* inv = nullptr;        // path order -> sorted
    uint64_t* qs = nullptr;        // sorted packed quantised positions
    uint32_t* redo = nullptr;      // kNN queries handed to the exact search
    uint32_t* nredo = nullptr;
};

void carve_grid(Carver& cv, GridBufs& g, int64_t N, int shift);
hipError_t run_grid(const pg_paths* p, GridBufs& g, VRec* rec, hipStream_t s, VRec* recp = nullptr);
hipError_t launch_gather_records(int64_t N, const int32_t* perm, const VRec* recp, VRec* rec, hipStream_t s);

// The cluster neighbour relation (pg_clusters.hip).  Arrays indexed by a
// sorted id unless noted; "position" is the place in cluster order.
struct ClusterBufs {
    int K = 0;                       // expected cluster size (the k parameter)
    int bits = 0;                    // centre grid: 2^bits cells per axis
    int64_t ncells = 0;
    unsigned long long* kmin = nullptr;   // min (key << 32 | path id)
    unsigned long long* nedge = nullptr;  // sum of the squared cluster sizes (graph export)
    unsigned long long* part = nullptr;   // per-block partials of the two reductions
    int32_t* live = nullptr;         // [0] = 1, [r+1]: round r split a cluster
    uint32_t* gcount = nullptr;      // centre grid: counts, then starts
    uint32_t* gpart = nullptr;
    uint32_t* gcell = nullptr;       // by sorted id (centres only): grid cell, rank in it
    uint32_t* grank = nullptr;
    uint64_t* gq = nullptr;          // centres in grid order: packed position,
    int32_t* gs = nullptr;           //   sorted id
    int32_t* gpid = nullptr;         //   path id
    int32_t* cid = nullptr;          // sorted id of the vertex's centre
    uint32_t* ccount = nullptr;      // members per centre [N+1]
    uint32_t* cstart = nullptr;      // first member of each centre's group [N+1]
    uint32_t* cpart = nullptr;
    uint32_t* cfill = nullptr;
    int32_t* members = nullptr;      // sorted ids grouped by centre
    uint32_t* mslot = nullptr;       // each vertex's slot in members
    unsigned long long* mkey = nullptr;   // by slot: key << 32 | path id
    uint64_t* mq = nullptr;          // by slot: packed quantised position
    uint8_t* newc = nullptr;         // by slot: new centre in the current split round
    uint32_t* nsplit = nullptr;      // [r]: clusters split in round r
    int32_t* splitlist = nullptr;    // their centres (sorted ids), one round at a time
    int32_t* stage_m = nullptr;      // by slot: staging of members, mkey and mq while a
    unsigned long long* stage_k = nullptr;   //   split cluster is regrouped in place
    uint64_t* stage_q = nullptr;
    int32_t* cperm = nullptr;        // position -> sorted id
    int32_t* cinv = nullptr;         // path id -> position
    uint2* crange = nullptr;         // position -> [first, end) position of its cluster
};
void carve_clusters(Carver& cv, ClusterBufs& cb, int64_t N, int K);
hipError_t run_clusters(const pg_paths* p, GridBufs& g, ClusterBufs& cb, hipStream_t s);
hipError_t launch_centre_out(int64_t N, const GridBufs& g, const ClusterBufs& cb, int32_t* out, hipStream_t s);

// Per-vertex data of the render in cluster order.
struct ClusterRender {
    VRec* crec = nullptr;      // records
    float4* tq = nullptr;      // (arriving direction, albedo)
    float4* wq = nullptr;      // (continuation direction, 1 / M+ of it)
    float* mp = nullptr;       // M+ + C p_e
    float* me = nullptr;       // Me of the environment sample
    float* y2 = nullptr;       // second aggregation buffer [N*3]
    uint32_t* rowlen = nullptr;   // export: row lengths, then row starts [N+1]
    uint32_t* rowpart = nullptr;
};
void carve_cluster_render(Carver& cv, ClusterRender& cr, int64_t N);

// Every buffer of one render in the internal (spatially sorted) order.
struct RenderBufs {
    GridBufs g;
    int64_t N = 0, P = 0;
    int K = 0, D = 0, schedule = 0;
    int tile = 0, tile_group = 0;   // launch shape of the propagation kernels
    bool tape = false;
    VRec* rec = nullptr;
    VRec* recp = nullptr;     // [N] the records in path order (grid build scratch)
    int32_t* col = nullptr;   // [ell_size(N, K)] sorted ids, sliced ELL
    float* w = nullptr;       // [ell_size(N, K)]
    float* gw = nullptr;      // [ell_size(N, K)] dw/dg (tape)
    float* b = nullptr;       // [N*3]
    float* dpt = nullptr;     // [N*3]
    float* r = nullptr;       // [N]
    float* alpha = nullptr;   // [N]
    int32_t* succ = nullptr;  // [N]
    int32_t* pred = nullptr;  // [N] (tape)
    float* x = nullptr;       // [N*3]
    float* y = nullptr;       // [N*3]
    int16_t* c16 = nullptr;   // compact ids of the two-pass aggregation (c16_row_sum)
    uint32_t* c16_base = nullptr;   // [n_slices + 1]
    uint32_t* c16_cnt = nullptr;    // [n_slices] scratch of the build
    uint32_t* c16_part = nullptr;   // scan partials
    int32_t* c16_ovf = nullptr;     // [ell_size] escaped ids
    int32_t* mcol = nullptr;  // shifted schedule
    float* mw = nullptr;
    float* c = nullptr;
    float* traj = nullptr;    // [(D+1)*N*3] (tape)
    float* zt = nullptr;      // [D*N*6] neighbour sums z_t and dz_t/dg per iteration (tape + PG_FLAG_STORE_Z)
    bool clusters = false;    // cluster neighbour relation: the render runs in cluster order
    ClusterBufs cl;
    ClusterRender cr;
};

// The taped two-pass aggregation that also stores z and dz/dg (zt, six floats
// per row) for the reverse sweep (pg_backward.hip); K4 in {8, 12, 16}.
hipError_t launch_spmv_c16_tape(int64_t N, int K, const int16_t* c16, const uint32_t* c16_base, const int32_t* ovf,
                                const float* w, const float* gw, const float* x, const float* b, const float* alpha,
                                float* y, float* zt, hipStream_t s, int tile, int tile_group);

// Reverse-mode buffers, carved right after a render's tape.
// Window of the transposed operator's in-degree ordering (vertices).
constexpr int kTWinBits = 7;
constexpr int kTWin = 1 << kTWinBits;

struct BackBufs {
    int64_t n_rows = 0, n_edge = 0, n_out = 0, n_slots = 0;   // dL/dg partial-sum slots
    float* lam_a = nullptr;    // adjoint of L_t, ping
    float* lam_b = nullptr;    // pong
    float* zbar = nullptr;     // [N*3]
    float* abar = nullptr;     // [N] d/d albedo
    float* bbar = nullptr;     // [N*3]
    float* dptbar = nullptr;   // [N*3]
    float* rbar = nullptr;     // [N]
    // W^T as sliced ELL (slices of 64 T-rows, at most cap entries per T-row),
    // T-rows ordered by in-degree within windows of kTWin vertices
    uint32_t cap = 0;
    int64_t nslices = 0;
    uint32_t* tdeg = nullptr;  // in-degree [N+1]
    uint32_t* tlen = nullptr;  // slice lengths [nslices+1]
    uint8_t* trank = nullptr;  // arrival rank of each edge at its T-row [ell_size(N, K)]
    uint32_t* soff = nullptr;  // slice offsets [nslices+1]
    int32_t* trow = nullptr;   // position -> vertex [N rounded up to kTWin]
    int32_t* tpos = nullptr;   // vertex -> position [N]
    int32_t* ppred = nullptr;  // position of each row's predecessor, -1: none [N]
    uint32_t* tpart = nullptr; // scan partials
    uint2* tent = nullptr;     // [nslices*64*cap] (source row, weight bits)
    int32_t* ovf = nullptr;    // overflow (j, i) pairs [2E]
    float* ovw = nullptr;      // overflow weights [E]
    uint32_t* novf = nullptr;
    double* gpart = nullptr;   // [n_slots]
    double* gchunk = nullptr;   // per-chunk totals of gpart
    float* image = nullptr;    // forward image when the tape is recomputed
    int32_t* cpid = nullptr;   // cluster relation: position -> path id
};
void carve_back(Carver& cv, BackBufs& bb, const RenderBufs& r, const pg_paths* p);
hipError_t run_backward(const pg_paths* p, const pg_params* q, RenderBufs& r, BackBufs& bb, const float* gimg,
                        float* grad_grid, float* grad_alpha, float* grad_g, hipStream_t s);

// The path tracer (pg_trace.hip).
int64_t tracer_paths(const pg_tracer* t);
size_t trace_ws_size(const pg_tracer* t);
hipError_t run_trace_count(const pg_tracer* t, int64_t* path_offsets, float* e_cam, void* ws, hipStream_t s);
hipError_t run_trace_write(const pg_tracer* t, const int64_t* path_offsets, const pg_records& o, void* ws,
                           hipStream_t s, int32_t** flag_out);

int resolve_schedule(const pg_params* q);
void carve_render(Carver& cv, RenderBufs& r, const pg_paths* p, const pg_params* q);
// The three phases of run_render: grid + kNN + edges + path pass (returns the
// buffer holding L_0), the D iterations (returns the buffer holding L_D), and
// the output to pixels.
hipError_t render_setup(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                        hipStream_t s, float** x0_out);
hipError_t render_iterate(RenderBufs& r, float* x0, hipStream_t s, float** final_x);
hipError_t render_output(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                         float* image, const float* cur, hipStream_t s);
// The same three phases with the cluster neighbour relation (cluster order).
hipError_t cluster_setup(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                         hipStream_t s, float** x0_out);
hipError_t cluster_iterate(RenderBufs& r, const pg_params* q, float* x0, hipStream_t s, float** final_x);
hipError_t cluster_output(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                          float* image, const float* cur, hipStream_t s);
// Reverse mode of the cluster relation (kernels in pg_clusters.hip).
hipError_t launch_cluster_cpid(int64_t N, const RenderBufs& r, int32_t* cpid, hipStream_t s);
hipError_t launch_cluster_out_adjoint(const pg_paths& P, const Consts& c, const RenderBufs& r, const float* gimg,
                                      float* abar, float* dptbar, float* rbar, float* lam, double* gpart,
                                      int64_t nblocks, hipStream_t s);
hipError_t launch_cluster_reverse_step(const RenderBufs& r, const pg_params* q, int t, const float* lam,
                                       float* lam_prev, float* abar, float* bbar, float* zbar, double* gpart,
                                       hipStream_t s);
hipError_t launch_cluster_edges_adjoint(const pg_paths& P, const Consts& c, const RenderBufs& r, const int32_t* cpid,
                                        const float* bbar, const float* dptbar, const float* rbar, float* abar,
                                        double* gpart, hipStream_t s);
// Runs grid, kNN, edges, paths, D iterations and pixels; fills `out` if given.
// *final_x receives the buffer holding L_D (sorted order).
hipError_t run_render(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out, float* image,
                      hipStream_t s, float** final_x = nullptr);

}  // namespace pg
