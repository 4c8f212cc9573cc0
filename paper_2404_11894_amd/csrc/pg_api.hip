// pg_api.hip -- the C ABI: argument validation, workspace layout and the
// order of kernel launches for each entry point.  Host code only.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "pg_api_common.h"

namespace pg {

thread_local std::string g_error;

pg_status fail(pg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

pg_status hip_fail(hipError_t e, const char* where) {
    return fail(PG_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

int32_t default_shift(int64_t N) {
    // the finest power-of-two grid with no more cells than vertices (about
    // one vertex per cell if they filled the unit cube; media fill less)
    int G = 1;
    while (G < 512 && (int64_t)(2 * G) * (2 * G) * (2 * G) <= N) G *= 2;
    int lg = 0;
    while ((1 << lg) < G) ++lg;
    return kQBits - lg;
}

pg_status validate_paths(const pg_paths* p, bool need_records) {
    if (!p) return fail(PG_ERR_ARG, "paths is NULL");
    if (p->n_vertices < 0 || p->n_vertices >= (int64_t)INT32_MAX)
        return fail(PG_ERR_ARG, "n_vertices = %lld out of range [0, 2^31-1)", (long long)p->n_vertices);
    if (p->width < 1 || p->height < 1 || p->spp < 1)
        return fail(PG_ERR_ARG, "width, height and spp must be >= 1");
    if (p->n_paths != (int64_t)p->width * p->height * p->spp)
        return fail(PG_ERR_ARG, "n_paths (%lld) != width * height * spp", (long long)p->n_paths);
    if (!p->path_offsets) return fail(PG_ERR_ARG, "path_offsets is NULL");
    if (!p->e_cam) return fail(PG_ERR_ARG, "e_cam is NULL");
    if (p->n_vertices > 0) {
        if (!p->pos || !p->dir_in || !p->dir_out) return fail(PG_ERR_ARG, "pos, dir_in and dir_out are required");
        if (need_records && (!p->l_sun || !p->dir_env || !p->l_env || !p->l_phase))
            return fail(PG_ERR_ARG, "l_sun, dir_env, l_env and l_phase are required");
        if (!p->albedo && !p->albedo_grid) return fail(PG_ERR_ARG, "albedo or albedo_grid is required");
    }
    if (p->albedo_grid && (p->albedo_grid_res < 1 || p->albedo_grid_res > 1024))
        return fail(PG_ERR_ARG, "albedo_grid_res must be in [1, 1024]");
    if (p->n_extra < 0 || p->n_extra > 1024) return fail(PG_ERR_ARG, "n_extra must be in [0, 1024]");
    if ((p->dir_pl == nullptr) != (p->l_pl == nullptr)) return fail(PG_ERR_ARG, "dir_pl and l_pl go together");
    if (p->n_extra > 0 && p->n_paths > 0 && (!p->fb_l_sun || !p->fb_dir_env || !p->fb_l_env))
        return fail(PG_ERR_ARG, "n_extra > 0 needs fb_l_sun, fb_dir_env and fb_l_env");
    return PG_OK;
}

pg_status validate_params(const pg_params* q) {
    if (!q) return fail(PG_ERR_ARG, "params is NULL");
    if (q->k < 1 || q->k > PG_MAX_K) return fail(PG_ERR_ARG, "k = %d outside [1, %d]", q->k, PG_MAX_K);
    if (q->D < 0 || q->D > (1 << 20)) return fail(PG_ERR_ARG, "D = %d outside [0, 2^20]", q->D);
    if (!(std::fabs(q->g) < 1.0f) || !(std::fabs(q->g_s) < 1.0f)) return fail(PG_ERR_ARG, "|g| and |g_s| must be < 1");
    if (!(q->env_pdf > 0.0f) || !std::isfinite(q->env_pdf)) return fail(PG_ERR_ARG, "env_pdf must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(q->sun_dir[a])) return fail(PG_ERR_ARG, "sun_dir must be finite");
    if (q->init != PG_INIT_PT && q->init != PG_INIT_ZERO) return fail(PG_ERR_ARG, "init must be PG_INIT_PT or PG_INIT_ZERO");
    if (q->final_gather != 0 && q->final_gather != 1) return fail(PG_ERR_ARG, "final_gather must be 0 or 1");
    if (q->cell_shift != 0 && (q->cell_shift < kMinShift || q->cell_shift > kQBits))
        return fail(PG_ERR_ARG, "cell_shift must be 0 or in [%d, %d]", kMinShift, kQBits);
    if (q->schedule < 0 || q->schedule > PG_SCHED_SCATTER) return fail(PG_ERR_ARG, "unknown schedule");
    if (q->tile != 0 && q->tile != 64 && q->tile != 128 && q->tile != 256 && q->tile != 512 && q->tile != 1024)
        return fail(PG_ERR_ARG, "tile = %d: 0, 64, 128, 256, 512 or 1024", q->tile);
    if (q->tile_group < 0 || q->tile_group > 65536) return fail(PG_ERR_ARG, "tile_group must be in [0, 65536]");
    if (q->flags & ~(PG_FLAG_CHECK | PG_FLAG_TAPE | PG_FLAG_EXACT_KNN | PG_FLAG_CLUSTERS | PG_FLAG_PERSISTENT |
                      PG_FLAG_STORE_Z))
        return fail(PG_ERR_ARG, "unknown flag bits");
    return PG_OK;
}

pg_status validate_clusters(const pg_paths* p, const pg_params* q) {
    if (!(q->flags & PG_FLAG_CLUSTERS)) return PG_OK;
    if (q->schedule != 0 && q->schedule != PG_SCHED_TWO_PASS)
        return fail(PG_ERR_UNSUPPORTED, "PG_FLAG_CLUSTERS runs the two-pass schedule only");
    if (p->n_vertices > 0 && !p->cluster_key) return fail(PG_ERR_ARG, "PG_FLAG_CLUSTERS needs paths->cluster_key");
    return PG_OK;
}

Consts make_consts(const pg_params* q, int K) {
    Consts c;
    c.rho = HG::make(q->g);
    c.pdf = HG::make(q->g_s);
    c.g = q->g;
    c.env_pdf = q->env_pdf;
    c.sun = f3{q->sun_dir[0], q->sun_dir[1], q->sun_dir[2]};
    c.K = K;
    c.init = q->init;
    c.final_gather = q->final_gather;
    return c;
}

pg_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return PG_OK;
    if (!ws) return fail(PG_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (((uintptr_t)ws & 255u) != 0) return fail(PG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(PG_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return PG_OK;
}

// pg_edges / pg_propagate / pg_gather take the k-nearest CSR of pg_knn.  The
// cluster relation's rows have other lengths, so its flag is refused on the
// host (no_clusters); with PG_FLAG_CHECK the caller's row_ptr is verified on
// the device (and the call returns) before any kernel reads col.
pg_status no_clusters(const pg_params* q) {
    if (q->flags & PG_FLAG_CLUSTERS)
        return fail(PG_ERR_UNSUPPORTED, "PG_FLAG_CLUSTERS: this call takes the k-nearest CSR of pg_knn (use "
                                        "pg_render for the cluster relation)");
    return PG_OK;
}

pg_status check_knn_layout(const pg_params* q, int64_t N, int K, const int64_t* row_ptr, int32_t* flag,
                           hipStream_t s) {
    if (!(q->flags & PG_FLAG_CHECK) || N == 0) return PG_OK;
    hipError_t e = launch_check_rows(N, K, row_ptr, flag, s);
    if (e != hipSuccess) return hip_fail(e, "check_rows");
    return finish(s, q, flag, q->flags);
}

pg_status finish(hipStream_t s, const pg_params* q, const int32_t* dflag, uint32_t flags) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (!(flags & PG_FLAG_CHECK) || !dflag) return PG_OK;
    (void)q;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int32_t h = 0;
    e = hipMemcpy(&h, dflag, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(flag)");
    if (h) {
        std::string m = "invalid device data:";
        if (h & kFlagPos) m += " position non-finite or outside [0,1];";
        if (h & kFlagOffsets) m += " path offsets not monotone or out of range;";
        if (h & kFlagIndex) m += " neighbour id out of range or row not starting with itself;";
        if (h & kFlagCluster) m += " a cluster has more than 4096 members (cluster_key not uniform?);";
        if (h & kFlagCapacity) m += " the cluster edges exceed out->edge_capacity (or 2^32);";
        if (h & kFlagRows) m += " row_ptr is not the k-nearest layout row_ptr[i] = i*K;";
        return fail(PG_ERR_INPUT, "%s", m.c_str());
    }
    return PG_OK;
}

// ------------------------------------------------------- grid / kNN plan ---

void carve_grid(Carver& cv, GridBufs& g, int64_t N, int shift) {
    const int G = 1 << (kQBits - shift);
    g.shift = shift;
    g.ncells = (int64_t)G * G * G;
    g.flag = cv.take<int32_t>(64);
    g.cells = cv.take<uint32_t>(g.ncells + 1);
    g.range = cv.take<uint2>(g.ncells);
    g.partials = cv.take<uint32_t>(scan_partials_bytes(g.ncells) / 4);
    g.cellid = cv.take<uint32_t>(N);
    g.rank = cv.take<uint32_t>(N);
    g.perm = cv.take<int32_t>(N);
    g.inv = cv.take<int32_t>(N);
    g.qs = cv.take<uint64_t>(N);
    g.redo = cv.take<uint32_t>(N);
    g.nredo = cv.take<uint32_t>(64);
}

// quantise, count, scan, scatter.  rec may be NULL; with recp the records are
// packed in path order first and gathered into the sorted order.
hipError_t run_grid(const pg_paths* p, GridBufs& g, VRec* rec, hipStream_t s, VRec* recp) {
    const int64_t N = p->n_vertices;
    hipError_t e;
    if ((e = launch_fill(g.flag, 64 * sizeof(int32_t), s)) != hipSuccess) return e;
    if ((e = launch_fill(g.cells, (size_t)(g.ncells + 1) * 4, s)) != hipSuccess) return e;
    if ((e = launch_quantize_count(N, p->pos, g.shift, g.cells, g.cellid, g.rank, g.flag, s)) != hipSuccess) return e;
    if ((e = launch_scan_exclusive(g.cells, g.cells, g.ncells, g.partials, s)) != hipSuccess) return e;
    if ((e = launch_cell_range(g.ncells, g.shift, g.cells, g.range, s)) != hipSuccess) return e;
    if (rec && recp) {
        if ((e = launch_pack_records(N, *p, recp, g.flag, s)) != hipSuccess) return e;
        if ((e = launch_scatter(N, *p, g.shift, g.cellid, g.rank, g.cells, g.perm, g.inv, g.qs, nullptr, s)) !=
            hipSuccess)
            return e;
        return launch_gather_records(N, g.perm, recp, rec, s);
    }
    return launch_scatter(N, *p, g.shift, g.cellid, g.rank, g.cells, g.perm, g.inv, g.qs, rec, s);
}

int shift_of(const pg_params* q, int64_t N) { return q && q->cell_shift ? q->cell_shift : default_shift(N); }

size_t propagate_size(const pg_paths* p, const pg_params* q) {
    const int64_t N = p->n_vertices;
    (void)q;
    Carver cv(nullptr);
    cv.take<int32_t>(64);
    cv.take<int32_t>(N);      // succ
    cv.take<float>(N);        // alpha
    cv.take<float>(3 * N);    // y
    return cv.size();
}

pg_status propagate_run(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                        const float* w_ind, const float* b, float* lplus, float* traj, void* ws, size_t ws_bytes,
                        hipStream_t s) {
    pg_status st;
    if ((st = validate_paths(paths, false)) || (st = validate_params(params)) || (st = no_clusters(params)))
        return st;
    const int64_t N = paths->n_vertices;
    if (N > 0 && (!row_ptr || !col || !w_ind || !b || !lplus))
        return fail(PG_ERR_ARG, "row_ptr, col, w_ind, b and lplus are required");
    if ((st = check_ws(ws, ws_bytes, propagate_size(paths, params)))) return st;
    const int K = (int)(N < params->k ? N : params->k);
    Carver cv(ws);
    int32_t* flag = cv.take<int32_t>(64);
    int32_t* succ = cv.take<int32_t>(N);
    float* alpha = cv.take<float>(N);
    float* y = cv.take<float>(3 * N);
    hipError_t e;
    if ((e = launch_fill(flag, 64 * 4, s)) != hipSuccess) return hip_fail(e, "fill");
    if ((st = check_knn_layout(params, N, K, row_ptr, flag, s))) return st;
    if (N == 0) return finish(s, params, flag, params->flags);
    if ((e = launch_fill_value(succ, (size_t)N * 4, 0xffffffffu, s)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_paths(paths->n_paths, N, paths->path_offsets, nullptr, nullptr, nullptr, nullptr, nullptr, PG_INIT_ZERO,
                          succ, nullptr, nullptr, flag, s)) != hipSuccess)
        return hip_fail(e, "paths");
    if ((e = launch_alpha(N, *paths, alpha, s)) != hipSuccess) return hip_fail(e, "alpha");
    for (int t = 1; t <= params->D; ++t) {
        if ((e = launch_spmv(N, K, col, w_ind, lplus, b, alpha, y, s)) != hipSuccess) return hip_fail(e, "spmv");
        if ((e = launch_shift(N, succ, y, lplus, s)) != hipSuccess) return hip_fail(e, "shift");
        if (traj && (e = hipMemcpyAsync(traj + (size_t)(t - 1) * N * 3, lplus, (size_t)N * 12,
                                        hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync");
    }
    return finish(s, params, flag, params->flags);
}

}  // namespace pg

using namespace pg;

extern "C" {

const char* pg_version(void) { return "pathgraph-gfx950 1.0.0"; }

const char* pg_last_error(void) { return g_error.c_str(); }

int32_t pg_default_cell_shift(int64_t n_vertices) { return default_shift(n_vertices < 0 ? 0 : n_vertices); }

// ------------------------------------------------------------------ kNN ---

static size_t knn_size(const pg_paths* p, int shift) {
    Carver cv(nullptr);
    GridBufs g;
    carve_grid(cv, g, p->n_vertices, shift);
    return cv.size();
}

pg_status pg_knn_workspace_size(const pg_paths* paths, int32_t k, int32_t cell_shift, size_t* bytes) {
    g_error.clear();
    pg_status st = validate_paths(paths, false);
    if (st) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    if (k < 1 || k > PG_MAX_K) return fail(PG_ERR_ARG, "k = %d outside [1, %d]", k, PG_MAX_K);
    if (cell_shift != 0 && (cell_shift < kMinShift || cell_shift > kQBits)) return fail(PG_ERR_ARG, "bad cell_shift");
    *bytes = knn_size(paths, cell_shift ? cell_shift : default_shift(paths->n_vertices));
    return PG_OK;
}

pg_status pg_knn(const pg_paths* paths, int32_t k, int32_t cell_shift, int64_t* row_ptr, int32_t* col, void* ws,
                 size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st = validate_paths(paths, false);
    if (st) return st;
    if (k < 1 || k > PG_MAX_K) return fail(PG_ERR_ARG, "k = %d outside [1, %d]", k, PG_MAX_K);
    if (cell_shift != 0 && (cell_shift < kMinShift || cell_shift > kQBits)) return fail(PG_ERR_ARG, "bad cell_shift");
    if (!row_ptr || (paths->n_vertices > 0 && !col)) return fail(PG_ERR_ARG, "row_ptr and col are required");
    const int64_t N = paths->n_vertices;
    const int K = (int)(N < k ? N : k);
    const int shift = cell_shift ? cell_shift : default_shift(N);
    hipStream_t s = (hipStream_t)stream;
    if ((st = check_ws(ws, ws_bytes, knn_size(paths, shift)))) return st;
    Carver cv(ws);
    GridBufs g;
    carve_grid(cv, g, N, shift);
    hipError_t e;
    if (N == 0) {
        if ((e = launch_fill(row_ptr, sizeof(int64_t), s)) != hipSuccess) return hip_fail(e, "fill");
        return finish(s, nullptr, nullptr, 0);
    }
    if ((e = run_grid(paths, g, nullptr, s)) != hipSuccess) return hip_fail(e, "grid build");
    e = launch_knn(N, K, shift, g.qs, g.perm, g.inv, g.range, nullptr, col, row_ptr, g.redo, g.nredo, false, s);
    if (e != hipSuccess) return hip_fail(e, "knn");
    return finish(s, nullptr, g.flag, 0);
}

// ---------------------------------------------------------------- trace ---

static pg_status validate_tracer(const pg_tracer* t) {
    if (!t) return fail(PG_ERR_ARG, "tracer is NULL");
    if (t->R < 1 || t->R > 4096) return fail(PG_ERR_ARG, "R = %d outside [1, 4096]", t->R);
    if (t->width < 1 || t->height < 1 || t->spp < 1 || t->max_depth < 1)
        return fail(PG_ERR_ARG, "width, height, spp and max_depth must be >= 1");
    if (t->crop_w && (t->crop_w < 1 || t->crop_h < 1 || t->crop_x0 < 0 || t->crop_y0 < 0 ||
                      t->crop_x0 + t->crop_w > t->width || t->crop_y0 + t->crop_h > t->height))
        return fail(PG_ERR_ARG, "invalid crop window");
    if (t->extra_samples < 0 || t->extra_samples > 1024) return fail(PG_ERR_ARG, "extra_samples must be in [0, 1024]");
    if (!(std::fabs(t->g) < 1.0) || !(t->majorant >= 0.0) || !std::isfinite(t->majorant))
        return fail(PG_ERR_ARG, "|g| < 1 and a finite majorant >= 0 are required");
    if (!t->sigma) return fail(PG_ERR_ARG, "sigma is NULL");
    const int64_t P = tracer_paths(t);
    if (P >= (int64_t)INT32_MAX) return fail(PG_ERR_ARG, "too many paths");
    if (P * (int64_t)t->max_depth >= (int64_t)UINT32_MAX)
        return fail(PG_ERR_UNSUPPORTED, "paths x max_depth must stay below 2^32 vertices");
    return PG_OK;
}

pg_status pg_trace_workspace_size(const pg_tracer* t, size_t* bytes) {
    g_error.clear();
    pg_status st = validate_tracer(t);
    if (st) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    *bytes = trace_ws_size(t);
    return PG_OK;
}

pg_status pg_trace_count(const pg_tracer* t, int64_t* path_offsets, int64_t* n_vertices, void* ws, size_t ws_bytes,
                         void* stream) {
    g_error.clear();
    pg_status st = validate_tracer(t);
    if (st) return st;
    if (!path_offsets || !n_vertices) return fail(PG_ERR_ARG, "path_offsets and n_vertices are required");
    if ((st = check_ws(ws, ws_bytes, trace_ws_size(t)))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = run_trace_count(t, path_offsets, nullptr, ws, s);
    if (e != hipSuccess) return hip_fail(e, "trace");
    if ((e = hipMemcpyAsync(n_vertices, path_offsets + tracer_paths(t), sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return PG_OK;
}

pg_status pg_trace_records(const pg_tracer* t, const int64_t* path_offsets, const pg_records* out, void* ws,
                           size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st = validate_tracer(t);
    if (st) return st;
    if (!path_offsets || !out) return fail(PG_ERR_ARG, "path_offsets and out are required");
    if (!out->pos || !out->dir_in || !out->dir_out || !out->albedo || !out->l_sun || !out->dir_env || !out->l_env ||
        !out->l_phase || !out->e_cam)
        return fail(PG_ERR_ARG, "every output array is required");
    if (t->extra_samples > 0 && (!out->fb_l_sun || !out->fb_dir_env || !out->fb_l_env))
        return fail(PG_ERR_ARG, "extra_samples > 0 needs fb_l_sun, fb_dir_env and fb_l_env");
    if ((t->pl_I[0] != 0.0 || t->pl_I[1] != 0.0 || t->pl_I[2] != 0.0) && (!out->dir_pl || !out->l_pl))
        return fail(PG_ERR_ARG, "a point light needs dir_pl and l_pl");
    if ((st = check_ws(ws, ws_bytes, trace_ws_size(t)))) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t* flag = nullptr;
    hipError_t e = run_trace_write(t, path_offsets, *out, ws, s, &flag);
    if (e != hipSuccess) return hip_fail(e, "trace");
    return finish(s, nullptr, flag, PG_FLAG_CHECK);
}

// ------------------------------------------------------------- clusters ---

static size_t clusters_size(const pg_paths* p, int32_t k, int shift) {
    Carver cv(nullptr);
    GridBufs g;
    carve_grid(cv, g, p->n_vertices, shift);
    ClusterBufs cb;
    carve_clusters(cv, cb, p->n_vertices, k);
    return cv.size();
}

pg_status pg_clusters_workspace_size(const pg_paths* paths, int32_t k, int32_t cell_shift, size_t* bytes) {
    g_error.clear();
    pg_status st = validate_paths(paths, false);
    if (st) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    if (k < 1 || k > PG_MAX_K) return fail(PG_ERR_ARG, "k = %d outside [1, %d]", k, PG_MAX_K);
    if (cell_shift != 0 && (cell_shift < kMinShift || cell_shift > kQBits)) return fail(PG_ERR_ARG, "bad cell_shift");
    *bytes = clusters_size(paths, k, cell_shift ? cell_shift : default_shift(paths->n_vertices));
    return PG_OK;
}

pg_status pg_clusters(const pg_paths* paths, int32_t k, int32_t cell_shift, int32_t* centre, void* ws,
                      size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st = validate_paths(paths, false);
    if (st) return st;
    if (k < 1 || k > PG_MAX_K) return fail(PG_ERR_ARG, "k = %d outside [1, %d]", k, PG_MAX_K);
    if (cell_shift != 0 && (cell_shift < kMinShift || cell_shift > kQBits)) return fail(PG_ERR_ARG, "bad cell_shift");
    const int64_t N = paths->n_vertices;
    if (N > 0 && (!centre || !paths->cluster_key)) return fail(PG_ERR_ARG, "centre and paths->cluster_key are required");
    const int shift = cell_shift ? cell_shift : default_shift(N);
    if ((st = check_ws(ws, ws_bytes, clusters_size(paths, k, shift)))) return st;
    hipStream_t s = (hipStream_t)stream;
    Carver cv(ws);
    GridBufs g;
    carve_grid(cv, g, N, shift);
    ClusterBufs cb;
    carve_clusters(cv, cb, N, k);
    if (N == 0) return finish(s, nullptr, nullptr, 0);
    hipError_t e;
    if ((e = run_grid(paths, g, nullptr, s)) != hipSuccess) return hip_fail(e, "grid build");
    if ((e = run_clusters(paths, g, cb, s)) != hipSuccess) return hip_fail(e, "clusters");
    if ((e = launch_centre_out(N, g, cb, centre, s)) != hipSuccess) return hip_fail(e, "centre output");
    return finish(s, nullptr, g.flag, PG_FLAG_CHECK);
}

// ---------------------------------------------------------------- edges ---

static size_t edges_size(const pg_paths* p, const pg_params* q, bool* ok) {
    const int64_t N = p->n_vertices;
    const int64_t K = N < q->k ? N : q->k;
    Carver cv(nullptr);
    cv.take<int32_t>(64);
    cv.take<VRec>(N);
    cv.take<float>(N * K);    // w if the caller does not want it
    cv.take<float>(3 * N);    // b
    cv.take<float>(3 * N);    // dpt
    cv.take<float>(N);        // r
    cv.take<float>(N);        // alpha
    *ok = true;
    return cv.size();
}

pg_status pg_edges_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params))) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    bool ok;
    *bytes = edges_size(paths, params, &ok);
    return PG_OK;
}

pg_status pg_edges(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                   float* w_ind, float* w_ph, float* w_env, float* b, float* d_pt, float* lplus0, void* ws,
                   size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params)) || (st = no_clusters(params)))
        return st;
    const int64_t N = paths->n_vertices;
    if (N > 0 && (!row_ptr || !col)) return fail(PG_ERR_ARG, "row_ptr and col are required");
    bool ok;
    if ((st = check_ws(ws, ws_bytes, edges_size(paths, params, &ok)))) return st;
    const int K = (int)(N < params->k ? N : params->k);
    hipStream_t s = (hipStream_t)stream;
    Carver cv(ws);
    int32_t* flag = cv.take<int32_t>(64);
    VRec* rec = cv.take<VRec>(N);
    float* wtmp = cv.take<float>(N * K);
    float* bl = cv.take<float>(3 * N);
    float* dl = cv.take<float>(3 * N);
    float* rl = cv.take<float>(N);
    float* al = cv.take<float>(N);
    hipError_t e;
    if ((e = launch_fill(flag, 64 * 4, s)) != hipSuccess) return hip_fail(e, "fill");
    if ((st = check_knn_layout(params, N, K, row_ptr, flag, s))) return st;
    if (N == 0) return finish(s, params, flag, params->flags);
    if ((e = launch_pack_records(N, *paths, rec, flag, s)) != hipSuccess) return hip_fail(e, "pack");
    EdgeOut o{};
    o.w = w_ind ? w_ind : wtmp;
    o.b = bl;
    o.dpt = dl;
    o.r = rl;
    o.alpha = al;
    o.w_ph = w_ph;
    o.w_env = w_env;
    o.b_canon = b;
    o.dpt_canon = d_pt;
    o.emit = paths->l_emit;
    o.dir_pl = paths->dir_pl;
    o.l_pl = paths->l_pl;
    Consts c = make_consts(params, K);
    if ((e = launch_edges(N, c, col, rec, o, flag, s)) != hipSuccess) return hip_fail(e, "edges");
    if (lplus0) {
        if ((e = launch_fill(lplus0, (size_t)N * 12, s)) != hipSuccess) return hip_fail(e, "fill");
        if ((e = launch_paths(paths->n_paths, N, paths->path_offsets, nullptr, al, dl, rl, paths->l_emit, params->init, nullptr,
                              nullptr, lplus0, flag, s)) != hipSuccess)
            return hip_fail(e, "paths");
    }
    return finish(s, params, flag, params->flags);
}

// ------------------------------------------------------------ propagate ---

pg_status pg_propagate_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, false)) || (st = validate_params(params))) return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    *bytes = propagate_size(paths, params);
    return PG_OK;
}

pg_status pg_propagate(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                       const float* w_ind, const float* b, float* lplus, float* traj, void* ws, size_t ws_bytes,
                       void* stream) {
    g_error.clear();
    return propagate_run(paths, params, row_ptr, col, w_ind, b, lplus, traj, ws, ws_bytes, (hipStream_t)stream);
}

// --------------------------------------------------------------- gather ---

pg_status pg_gather(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                    const float* w_ind, const float* d_pt, const float* lplus, float* image, void* stream) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, false)) || (st = validate_params(params))) return st;
    if (!image) return fail(PG_ERR_ARG, "image is NULL");
    const int64_t N = paths->n_vertices;
    if (N > 0 && (!row_ptr || !col || !w_ind || !d_pt || !lplus))
        return fail(PG_ERR_ARG, "row_ptr, col, w_ind, d_pt and lplus are required");
    if (params->flags & PG_FLAG_CHECK) return fail(PG_ERR_UNSUPPORTED, "pg_gather has no workspace for PG_FLAG_CHECK");
    if ((st = no_clusters(params))) return st;
    const int K = (int)(N < params->k ? N : params->k);
    hipStream_t s = (hipStream_t)stream;
    Consts c = make_consts(params, K);
    hipError_t e = launch_pixels(*paths, c, nullptr, col, w_ind, lplus, d_pt, nullptr, nullptr, image, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "pixels");
    return finish(s, params, nullptr, 0);
}

// --------------------------------------------------------------- render ---

pg_status pg_render_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params)) || (st = validate_clusters(paths, params)))
        return st;
    if (!bytes) return fail(PG_ERR_ARG, "bytes is NULL");
    Carver cv(nullptr);
    RenderBufs r;
    carve_render(cv, r, paths, params);
    if (params->flags & PG_FLAG_TAPE) {
        // room for the reverse pass too, so one workspace serves pg_render and pg_backward
        BackBufs bb;
        carve_back(cv, bb, r, paths);
    }
    *bytes = cv.size();
    return PG_OK;
}

pg_status pg_render(const pg_paths* paths, const pg_params* params, float* image, const pg_graph_out* out, void* ws,
                    size_t ws_bytes, void* stream) {
    g_error.clear();
    pg_status st;
    if ((st = validate_paths(paths, true)) || (st = validate_params(params)) || (st = validate_clusters(paths, params)))
        return st;
    if (!image) return fail(PG_ERR_ARG, "image is NULL");
    Carver dry(nullptr);
    RenderBufs r;
    carve_render(dry, r, paths, params);
    if ((st = check_ws(ws, ws_bytes, dry.size()))) return st;
    Carver cv(ws);
    carve_render(cv, r, paths, params);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = run_render(paths, params, r, out, image, s);
    if (e != hipSuccess) return hip_fail(e, "render");
    // the cluster relation always reports its device checks (one synchronisation)
    const uint32_t fl = r.clusters ? params->flags | PG_FLAG_CHECK : params->flags;
    return finish(s, params, r.g.flag, fl);
}

}  // extern "C"
