/*
 * pathgraph.h -- C ABI of the MI355X (gfx950) path-graph library.
 *
 * The library implements the data-parallel hot path of path-graph rendering
 * for participating media (Hu, Deng, Luan, Hasan, Marschner, arXiv
 * 2404.11894): from the volume path vertices a path tracer recorded, it builds
 * the path graph (neighbour search), turns each vertex's neighbours into
 * weighted edges (aggregation operators), iterates aggregation + propagation
 * D times and writes the radiance of every path's first continuation edge
 * into its pixel.  It also provides the reverse-mode derivative of an image
 * objective with respect to a trilinear albedo grid and the HG parameter, and
 * a batched render of many independent scenes.
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller; the
 *   library never allocates, frees or retains it.  Temporary memory is a
 *   caller-provided device workspace of at least the size the matching
 *   *_workspace_size call reports (256-byte alignment required).  The library
 *   keeps no state between calls except a thread-local error string.
 * Streams.  `stream` is a hipStream_t (NULL: the null stream).  Calls enqueue
 *   work and return; results are ready when the stream is.  With
 *   PG_FLAG_CHECK in params->flags a call synchronises the stream and reports
 *   input errors detected on the device as PG_ERR_INPUT.
 * Errors.  Every call returns a pg_status.  On error the outputs are
 *   undefined and pg_last_error() describes the cause.  No C++ exception
 *   crosses the interface.  Bad device data (NaN or out-of-range positions,
 *   non-monotone path offsets, neighbour ids out of range) never causes an
 *   out-of-bounds access: the offending item is skipped and a device flag set.
 * Layout.  Per-vertex arrays are in PATH ORDER (the order the path tracer
 *   recorded the vertices, paper Sec. "Rendering System", instrumented path
 *   tracer).  float3 data is packed [N][3].  Vertex ids are int32, so N must be
 *   below 2^31; path offsets and CSR row pointers are int64.
 * Threading.  Calls on different streams/workspaces may run concurrently.
 */
#ifndef PATHGRAPH_H
#define PATHGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pg_status;
#define PG_OK               0
#define PG_ERR_ARG         -1   /* invalid argument (null pointer, size, range) */
#define PG_ERR_WORKSPACE   -2   /* workspace missing, too small or misaligned */
#define PG_ERR_HIP         -3   /* a HIP runtime call failed */
#define PG_ERR_INPUT       -4   /* bad device data detected (PG_FLAG_CHECK) */
#define PG_ERR_UNSUPPORTED -5   /* valid request the library does not support */

#define PG_INIT_PT   0  /* start from the path tracer's own incoming-indirect estimate */
#define PG_INIT_ZERO 1  /* start the indirect part from zero (L+_0 = the emission collected at
                           the successor, 0 without l_emit) */

#define PG_FLAG_CHECK 1u  /* synchronise and report device-detected input errors */
#define PG_FLAG_TAPE  2u  /* pg_render keeps the graph and every iterate in the workspace
                             for a following pg_backward on the same workspace */
#define PG_FLAG_EXACT_KNN 4u  /* every neighbour query takes the exact (d^2, id) search instead
                                 of the packed-key fast path: the same neighbours, slower; for
                                 validating the fallback the fast path hands rare queries to */
#define PG_FLAG_CLUSTERS 8u  /* pg_render / pg_backward: neighbours are the disjoint clusters of
                                pg_clusters (k = expected cluster size) instead of the k nearest.
                                Two-pass schedule only.  pg_render, pg_backward and
                                pg_render_batched synchronise once to report device checks (a
                                pg_batch plan does not report them). */

#define PG_FLAG_PERSISTENT 16u  /* pg_render_batched / pg_batch_create (read from the first scene's
                                   params; ignored by the other calls): all D iterations of all
                                   scenes run as ONE cooperative kernel with grid barriers between
                                   the aggregation and the shift, instead of one aggregation and one
                                   shift launch per iteration.  Same results bit for bit; slower on
                                   MI355X (every barrier is a device-scope release and acquire by
                                   every workgroup across the XCDs' separate L2 caches).  Needs
                                   tile 0 or 256.  pg_render_batched reports a timed-out barrier
                                   as PG_ERR_HIP; a pg_batch plan does not check. */

#define PG_FLAG_STORE_Z 32u  /* with PG_FLAG_TAPE (pg_render, and pg_backward, which sets the tape
                                itself): the forward also keeps every iteration's neighbour sums
                                z_t = W x_(t-1) and dz_t/dg (6 floats per vertex per iteration,
                                24 D N bytes more workspace), so the reverse sweep reads them
                                instead of gathering x_(t-1) again.  Same gradients bit for bit.
                                Taken when the two-pass schedule runs on the compact ids with
                                K rounded up to 8, 12 or 16; otherwise no effect. */

#define PG_SCHED_TWO_PASS 1  /* aggregate over spatially sorted rows, then shift along paths */
#define PG_SCHED_SHIFTED  2  /* rows pre-arranged in predecessor order: one pass per iteration */
#define PG_SCHED_SCATTER  3  /* sorted rows; each writes its result straight to its predecessor */

#define PG_MAX_K 64

/* The recorded paths of one image (paper Sec. "Path Graph Framework": a path
 * graph is built from complete light paths sampled at one or more samples per
 * pixel; all samples of the image go into one graph).
 * Path p = vertices [path_offsets[p], path_offsets[p+1]) belongs to pixel
 * p / spp (row-major, width fastest), sample p % spp.  An empty path is a
 * camera ray that escaped; inside a path, vertex v+1 is the successor of v. */
typedef struct pg_paths {
    int64_t n_vertices;           /* N */
    int64_t n_paths;              /* P = width * height * spp */
    int32_t width, height, spp;
    int32_t albedo_grid_res;      /* R of albedo_grid, 0 if none */
    const int64_t* path_offsets;  /* [P+1], path_offsets[0] = 0, path_offsets[P] = N */
    const float* pos;             /* [N][3] collision position in [0,1]^3 */
    const float* dir_in;          /* [N][3] unit travel direction of the path arriving at v */
    const float* dir_out;         /* [N][3] unit continuation direction, sampled from HG(g_s) about dir_in */
    const float* albedo;          /* [N] scattering albedo sigma_s / sigma_t at v (ignored with a grid) */
    const float* l_sun;           /* [N][3] sun NEE: sun irradiance x shadow-ray transmittance */
    const float* dir_env;         /* [N][3] unit environment NEE direction (pdf env_pdf) */
    const float* l_env;           /* [N][3] environment radiance x shadow-ray transmittance */
    const float* l_phase;         /* [N][3] environment radiance if the continuation escaped, else 0 */
    const float* e_cam;           /* [P][3] environment radiance if the camera ray escaped, else 0 */
    const float* albedo_grid;     /* [R][R][R] (z,y,x) or NULL: albedo = cell-centred trilinear
                                     interpolation of the grid at pos (indices clamped to [0,R-1]) */
    const float* l_emit;          /* [N][3] or NULL (no emission): volume emission at v divided by
                                     sigma_t(v), the delta-tracking estimate of the emission term of
                                     the RTE (Sec. "Radiative Transfer Equation in a Medium", the
                                     operator G applied to the volume emission).  It is radiance that
                                     leaves v toward its predecessor unscattered: it is added to the
                                     constant b_v, to the path-traced L+_0 of the predecessor and, at
                                     a path's first vertex, to the pixel.  A constant input: the
                                     reverse mode does not differentiate it. */
    const uint32_t* cluster_key;  /* [N] or NULL: uniform random 32-bit keys drawn by the caller, one
                                     per vertex; they choose the cluster centres of pg_clusters and of
                                     PG_FLAG_CLUSTERS (required there) */
    /* Extra emitter samples at each path's first vertex (Sec. "Rendering System", handling
     * direct light), [P][n_extra][3] each, zero for a path without vertices: with n_extra > 0
     * the pixel uses their estimate (1/M) sum_m (rho(sun) l_sun_m + rho(we_m) l_env_m / env_pdf)
     * in place of the first vertex's d_pt; the propagation is unchanged. */
    const float* fb_l_sun;        /* sun irradiance x shadow-ray transmittance */
    const float* fb_dir_env;      /* unit uniform-sphere environment directions */
    const float* fb_l_env;        /* environment radiance x shadow-ray transmittance */
    int32_t n_extra;              /* M, 0..1024; 0: none (the three pointers are ignored) */
    int32_t pad_;
    /* A point light (a delta light whose direction differs per vertex; more light types enter
     * only the constant terms): [N][3] each, both or neither.  Like the sun it takes no MIS:
     * d_agg_i += (1/K) sum_j rho_i(dir_pl_j) l_pl_j and d_pt_i += rho_i(dir_pl_i) l_pl_i. */
    const float* dir_pl;          /* unit direction toward the light */
    const float* l_pl;            /* intensity x shadow-ray transmittance / distance^2 */
} pg_paths;

/* Method parameters. */
typedef struct pg_params {
    int32_t k;              /* neighbours per vertex, the vertex itself included; 1..PG_MAX_K.
                               K = min(k, N) */
    int32_t D;              /* aggregation + propagation iterations, >= 0 */
    float g;                /* HG parameter of the receiver's phase function, |g| < 1 */
    float g_s;              /* HG parameter of the sampling pdfs in the MIS marginals, |g_s| < 1 */
    float sun_dir[3];       /* unit direction toward the (delta) sun */
    float env_pdf;          /* solid-angle pdf of environment sampling, > 0 (1/(4 pi)) */
    int32_t init;           /* PG_INIT_PT or PG_INIT_ZERO */
    int32_t final_gather;   /* 0: the first vertex aggregates its neighbours' radiance for the
                               output; 1: it uses its own continuation sample only */
    int32_t cell_shift;     /* uniform-grid cell = 2^cell_shift quantisation steps per axis,
                               11..20; 0 = choose from N */
    int32_t schedule;       /* propagation schedule, same result: 0 = default,
                               PG_SCHED_TWO_PASS, PG_SCHED_SHIFTED or PG_SCHED_SCATTER */
    uint32_t flags;         /* PG_FLAG_* */
    /* Launch shape of the propagation kernels (pg_render's iterations and the
     * batched ones); any value gives bit-identical results.  0 = default. */
    int32_t tile;           /* workgroup size of the aggregation (one row per thread) and the
                               shift (two vertices per thread): 64, 128, 256, 512 or 1024;
                               default 512 in pg_render and its reverse mode, 256 in a batch
                               (the first scene's params set the batch's tile); pg_propagate's
                               path-order product has a fixed shape */
    int32_t tile_group;     /* consecutive row tiles each XCD takes in turn in the aggregation
                               (the hardware hands workgroup b to XCD b mod 8): 1 (default) =
                               plain launch order, G > 1 = tiles [8Gc + Gx, 8Gc + G(x + 1)) go
                               to XCD x; at most 65536 */
} pg_params;

/* Optional outputs of pg_render; any pointer may be NULL. */
typedef struct pg_graph_out {
    int64_t* row_ptr;       /* [N+1]  = i*K (clusters: row i = its cluster's members) */
    int32_t* col;           /* [E]    neighbour ids (path-order ids); E = N*K, or with
                               PG_FLAG_CLUSTERS the sum over clusters of size^2, ids ascending */
    float* w_ind;           /* [E]    indirect aggregation weights */
    float* w_ph;            /* [E]    direct weights of the phase-sampled records */
    float* w_env;           /* [E]    direct weights of the emitter-sampled records */
    float* b;               /* [N][3] albedo x aggregated direct radiance */
    float* d_pt;            /* [N][3] non-aggregated (path-traced) direct term */
    float* lplus;           /* [N][3] incoming indirect radiance after D iterations */
    int64_t edge_capacity;  /* PG_FLAG_CLUSTERS: entries col / w_* hold; a larger E writes no
                               edges and returns PG_ERR_INPUT (E from pg_clusters' centres) */
    int64_t* n_far;         /* [1]    edges whose neighbour lies more than 32767 rows from its
                               row in the spatially sorted order the iterations run in (their
                               ids are read from a side list, 4 more bytes each); 0 when the
                               iterations do not use the compact 16-bit ids */
} pg_graph_out;

/* ---- utilities ---------------------------------------------------------- */

/* Library version string (static storage). */
const char* pg_version(void);

/* Text of the last error raised on the calling thread ("" if none). */
const char* pg_last_error(void);

/* Cell shift chosen when params->cell_shift == 0, for N vertices. */
int32_t pg_default_cell_shift(int64_t n_vertices);

/* ---- instrumentation ------------------------------------------------------
 * Between pg_profile_start and pg_profile_stop, every kernel step that calls
 * on the calling thread enqueue is bracketed by two HIP events recorded on
 * the caller's stream.  pg_profile_stop waits for the events, aggregates the
 * elapsed times by step name into out[0 .. *n_entries-1] (at most
 * max_entries) and stops recording.  Off by default; costs two event records
 * per step when on. */
typedef struct pg_profile_entry {
    char name[32];        /* step, e.g. "spmv", "shift", "knn", "edges" */
    int32_t count;        /* launches recorded */
    double total_ms;      /* summed event-to-event time */
    double max_ms;
} pg_profile_entry;
pg_status pg_profile_start(void);
pg_status pg_profile_stop(int32_t max_entries, pg_profile_entry* out, int32_t* n_entries);

/* ---- step 1: path graph neighbour edges ---------------------------------
 * Paper Sec. "Path Graph Framework" (neighbour edges connect each shading
 * point with the points in its spatial neighbourhood) and Sec. "Rendering
 * System" (a hash grid over the shading points and a search through
 * neighbouring bins).  Neighbourhoods here are exact k nearest neighbours on
 * positions quantised to 20 bits per axis, q = min(floor(x * 2^20), 2^20-1):
 * row i lists i first, then the K-1 nearest j != i ordered by (squared integer
 * distance, j).  The result is unique and reproducible bit for bit.
 * Writes row_ptr[N+1] (= i*K) and col[N*K]. */
pg_status pg_knn_workspace_size(const pg_paths* paths, int32_t k, int32_t cell_shift, size_t* bytes);
pg_status pg_knn(const pg_paths* paths, int32_t k, int32_t cell_shift, int64_t* row_ptr, int32_t* col,
                 void* ws, size_t ws_bytes, void* stream);

/* ---- upstream: the instrumented path tracer --------------------------------
 * Paper Sec. "Volume Path Tracing" and Sec. "Rendering System" (instrumented
 * path tracer), on the GPU: traces every path of a (cropped) image through a
 * grid medium and writes the path-ordered vertex records that pg_paths
 * describes, in HBM.  Medium: extinction sigma on an R^3 grid over [0,1]^3
 * (nearest voxel, x fastest), vacuum outside; albedo per voxel or constant.
 * Lights: a directional (delta) sun and a constant environment.  Per path: a
 * jittered camera ray, analog delta tracking against `majorant`; at every
 * collision a sun shadow ray and one uniform-sphere environment shadow ray
 * (ratio-tracking transmittance) and a continuation sampled from HG(g) about
 * the arriving direction; at most max_depth vertices; no Russian roulette.
 * Random numbers: PCG32, one stream per pixel of the full image, seeded from
 * (seed, sample) through splitmix64 (the pixel jitter takes the stream's
 * first two numbers, y first; sphere and HG samples draw the azimuth number
 * first).  Double precision, no contraction.  Paths are numbered pixel-major
 * over the crop window, spp consecutive paths per pixel. */
typedef struct pg_tracer {
    int32_t R;                 /* grid resolution per axis */
    int32_t width, height;     /* full image */
    int32_t spp, max_depth;
    int32_t crop_x0, crop_y0, crop_w, crop_h;   /* traced window; crop_w == 0: full image */
    int32_t extra_samples;     /* M extra emitter samples at each path's first vertex, 0..1024,
                                  from a second stream per pixel (the paths do not depend on M) */
    const float* sigma;        /* [R^3] device: extinction coefficients */
    const float* albedo;       /* [R^3] device, or NULL: albedo_const everywhere */
    double albedo_const;
    double majorant;           /* >= every sigma (the grid maximum); 0: no medium */
    double g;                  /* HG parameter of the continuation sampling */
    double cam_pos[3], look_at[3], vfov_deg;   /* pinhole camera, world up +y */
    double sun_dir[3];         /* unit vector toward the sun */
    double sun_E[3];           /* sun irradiance */
    double env_L[3];           /* environment radiance */
    uint64_t seed;
    double pl_pos[3];          /* point light position (may be outside the cube) */
    double pl_I[3];            /* its intensity; all zero: no point light.  Its shadow ray
                                  (ratio tracking up to the light or the cube's exit) is drawn
                                  after the environment shadow ray */
} pg_tracer;

/* Device output arrays of pg_trace_records ([N][3], albedo [N], e_cam [P][3],
 * fb_* [P][M][3], required when extra_samples > 0, zero for an escaped path;
 * a point light's records). */
typedef struct pg_records {
    float *pos, *dir_in, *dir_out, *albedo, *l_sun, *dir_env, *l_env, *l_phase, *e_cam;
    float *fb_l_sun, *fb_dir_env, *fb_l_env;
    float *dir_pl, *l_pl;      /* [N][3], required with a point light */
} pg_records;

/* Pass 1: traces every path and writes path_offsets[P+1] (device); N to
 * *n_vertices (host; the call synchronises the stream once).  The records
 * stay in the workspace, which holds max_depth record slots per path
 * (about 88 bytes each, 24 more with a point light) plus the paths' extra
 * samples: pg_trace_workspace_size grows with P * max_depth. */
pg_status pg_trace_workspace_size(const pg_tracer* t, size_t* bytes);
pg_status pg_trace_count(const pg_tracer* t, int64_t* path_offsets, int64_t* n_vertices, void* ws,
                         size_t ws_bytes, void* stream);
/* Pass 2: copies the records pass 1 left in the workspace to the offsets
 * of pass 1 (same tracer settings; the workspace passed to pass 1, unchanged
 * since).  A path whose offsets do not span exactly its traced vertex count
 * is not written and the call returns PG_ERR_INPUT; no record is written
 * outside a path's slots.  Synchronises the stream once. */
pg_status pg_trace_records(const pg_tracer* t, const int64_t* path_offsets, const pg_records* out, void* ws,
                           size_t ws_bytes, void* stream);

/* ---- step 1, the paper's relation: clusters ---------------------------------
 * Paper Sec. "Path Graph Framework" (disjoint clusters of about K points
 * around randomly chosen centres, large clusters split again) and Sec.
 * "Rendering System" (path graph solver: centres chosen at random, nearest
 * centre through neighbouring bins of a grid).  Readings:
 *   - vertex i is a centre when cluster_key[i] < floor(2^32 / k), so about
 *     N/k of them; the vertex of smallest (key, id) always is one;
 *   - every vertex joins the nearest centre by (squared distance of the 20-bit
 *     quantised positions, centre id);
 *   - a cluster of s > 2k members takes its ceil(s/k) members of smallest
 *     (key, id) as new centres and its members join the nearest of those;
 *     up to 4 rounds, for the clusters still above 2k.
 * Writes centre[N] (path order): the id of the centre of each vertex's
 * cluster.  Requires paths->cluster_key.  Synchronises the stream once;
 * returns PG_ERR_INPUT if a cluster exceeds 4096 members (non-uniform keys). */
pg_status pg_clusters_workspace_size(const pg_paths* paths, int32_t k, int32_t cell_shift, size_t* bytes);
pg_status pg_clusters(const pg_paths* paths, int32_t k, int32_t cell_shift, int32_t* centre, void* ws,
                      size_t ws_bytes, void* stream);

/* ---- step 2: aggregation operators ---------------------------------------
 * Paper Sec. "Path Graph Operators", eqs. (indirect-weight), (ag-indirect),
 * (ag-direct).  For receiver i and neighbour j (K = row length):
 *   M+_ij = sum_{l in N(i)} p_l(w_j),  p_l = HG_{g_s} about dir_in[l]
 *   w_ind_ij = rho_i(w_j) / M+_ij,      rho_i = HG_g about dir_in[i]
 *   w_ph_ij  = rho_i(w_j) / (M+_ij + K env_pdf)
 *   w_env_ij = rho_i(we_j) / (sum_l p_l(we_j) + K env_pdf)
 *   b_i = e_i + albedo_i (rho_i(sun) mean_j l_sun_j + sum_j w_env_ij l_env_j + w_ph_ij l_phase_j
 *                         [+ mean_j rho_i(dir_pl_j) l_pl_j])
 *         (e = l_emit, 0 if NULL; the point-light term only with dir_pl / l_pl)
 *   d_pt_i = rho_i(sun) l_sun_i + rho_i(we_i) l_env_i / (p_i(we_i) + env_pdf)
 *            + rho_i(w_i) l_phase_i / (p_i(w_i) + env_pdf)
 * and the initial radiance arriving along the continuation, lplus0 (paper Sec.
 * "Rendering System": the path tracer's own estimate, or zero): for v with
 * successor u, lplus0(v) = e_u + albedo_u (d_pt_u + rho_u(w_u)/p_u(w_u) lplus0(u))
 * with PG_INIT_PT, e_u with PG_INIT_ZERO; 0 at a path's end.
 * Inputs row_ptr/col as produced by pg_knn (row i = [i K, (i+1) K), starting
 * with i); this call, pg_propagate and pg_gather read col and the weights at
 * i K + l.  PG_FLAG_CLUSTERS is refused with PG_ERR_UNSUPPORTED (cluster rows
 * have other lengths: pg_render handles that relation).  With PG_FLAG_CHECK,
 * row_ptr is verified on the device before col is read, and a row_ptr of any
 * other layout returns PG_ERR_INPUT; without it, such a row_ptr is the
 * caller's error.  Any of the outputs may be NULL. */
pg_status pg_edges_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes);
pg_status pg_edges(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                   float* w_ind, float* w_ph, float* w_env, float* b, float* d_pt, float* lplus0,
                   void* ws, size_t ws_bytes, void* stream);

/* ---- step 3: iterated aggregation and propagation ------------------------
 * Paper eqs. (ag-mf), (rte-pg), (rte-mff).  For t = 1..D:
 *   y_i = b_i + albedo_i sum_j w_ind_ij L(j);  L(v) = y(v+1) inside a path, 0 at its end.
 * (Under delta tracking the propagation factor transmittance / free-flight pdf
 * is 1/sigma_t at the collision, which turns sigma_s * phase into albedo *
 * phase, so propagation is the shift to the predecessor.)
 * lplus holds L_0 on entry and L_D on return.  traj, if not NULL, receives
 * L_1..L_D as [D][N][3].  row_ptr / col: the k-nearest layout, checked as in
 * pg_edges. */
pg_status pg_propagate_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes);
pg_status pg_propagate(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr,
                       const int32_t* col, const float* w_ind, const float* b, float* lplus, float* traj,
                       void* ws, size_t ws_bytes, void* stream);

/* ---- step 3 without allocation -------------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops, harnesses that forbid hipMalloc): pg_propagate with
 * the same arguments, results and errors, but no workspace argument.  Its
 * workspace is a static device array of PG_STATIC_SCRATCH_BYTES (64 MiB) that
 * the library holds on every GPU it runs on until the process ends; the call
 * allocates nothing.  It serves graphs whose pg_propagate_workspace_size is at
 * most that (20 bytes per vertex plus alignment: N up to about 3.3 million)
 * and returns PG_ERR_WORKSPACE for larger ones.  The array's address on the
 * current device (which must be the stream's) is looked up on the first call
 * there.  Every call on one GPU uses the same array, so calls that overlap in
 * time on one GPU (other streams, other threads) race and must be serialised
 * by the caller; each call initialises the parts it reads. */
#define PG_STATIC_SCRATCH_BYTES (64u << 20)
pg_status pg_propagate_static(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr,
                              const int32_t* col, const float* w_ind, const float* b, float* lplus, float* traj,
                              void* stream);

/* ---- step 4: output to pixels --------------------------------------------
 * Paper Sec. "Rendering System", "Handling direct Light" and "Final output":
 * path p with first vertex v0 outputs
 *   o_p = e_v0 + albedo_v0 (d_pt_v0 + sum_j w_ind_v0j L(j))        (final_gather = 0)
 *   o_p = e_v0 + albedo_v0 (d_pt_v0 + rho_v0(w_v0)/p_v0(w_v0) L(v0)) (final_gather = 1)
 * (0 for an empty path; d_pt_v0 replaced by the extra first-vertex samples'
 * estimate when paths->n_extra > 0) and image[pixel] = mean over its spp
 * paths of (e_cam_p + o_p).  image is [height][width][3].  No workspace, so
 * PG_FLAG_CHECK is refused; row_ptr / col: the k-nearest layout, as in
 * pg_edges (PG_FLAG_CLUSTERS refused). */
pg_status pg_gather(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr, const int32_t* col,
                    const float* w_ind, const float* d_pt, const float* lplus, float* image, void* stream);

/* ---- all four steps -------------------------------------------------------
 * pg_knn + pg_edges + pg_propagate + pg_gather in one call, with the graph
 * kept in a spatially sorted internal layout.  `out` may be NULL. */
pg_status pg_render_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes);
pg_status pg_render(const pg_paths* paths, const pg_params* params, float* image, const pg_graph_out* out,
                    void* ws, size_t ws_bytes, void* stream);

/* ---- reverse mode (project addition; not in the paper) --------------------
 * Gradient of  sum_px <grad_image[px], image[px]>  with respect to the albedo
 * grid (paths->albedo_grid, required) and the receiver-side HG parameter g,
 * with the recorded paths and the sampling pdfs (g_s) held fixed:
 * d rho/d g = rho * (-2g/(1-g^2) - 3(g - cos)/(1 + g^2 - 2 g cos)).
 * If params->flags has PG_FLAG_TAPE, `ws` must hold the tape of a pg_render
 * call with the same paths and params (PG_FLAG_TAPE set) and must not have
 * been used since; otherwise the forward pass is recomputed first.
 * grad_grid is [R][R][R]; grad_albedo ([N], per vertex) may be NULL;
 * grad_g is one float.  With PG_FLAG_CLUSTERS the tape holds x_0 and y_1..y_D
 * and the transposed product runs over each sample's own cluster. */
pg_status pg_backward_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes);
pg_status pg_backward(const pg_paths* paths, const pg_params* params, const float* grad_image,
                      float* grad_grid, float* grad_albedo, float* grad_g, void* ws, size_t ws_bytes,
                      void* stream);

/* ---- batching (project addition; not in the paper) ------------------------
 * Renders n_scenes independent scenes (each with its own paths and params;
 * k, D, g, cell size may differ) into images[s] ([height_s][width_s][3]).
 * The one-time steps run per scene; every one of the D iterations is one
 * aggregation launch and one shift launch for all scenes still iterating.
 * The result equals n_scenes pg_render calls (two-pass schedule).  The call
 * synchronises the stream once, after copying its small scene table. */
pg_status pg_render_batched_workspace_size(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                                           size_t* bytes);
pg_status pg_render_batched(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                            float* const* images, void* ws, size_t ws_bytes, void* stream);

/* A reusable batch: the same scenes rendered again and again (new input
 * VALUES in the same device arrays are picked up by every launch).  With
 * use_graph != 0 the whole sequence -- per-scene setup spread over four
 * streams, the batched iterations, per-scene output -- is captured once in a
 * hipGraph and every pg_batch_launch is a single graph launch.  The plan keeps
 * the pointers it was given (paths arrays, images, workspace), which must stay
 * valid and unchanged until pg_batch_destroy; it owns only host memory, three
 * streams, events and the graph.  The workspace size is
 * pg_render_batched_workspace_size's.  Launches of one plan must not overlap.
 * Capture needs a created stream (not the null stream). */
typedef struct pg_batch pg_batch;
pg_status pg_batch_create(int32_t n_scenes, const pg_paths* paths, const pg_params* params, float* const* images,
                          void* ws, size_t ws_bytes, int32_t use_graph, void* stream, pg_batch** plan);
pg_status pg_batch_launch(pg_batch* plan, void* stream);
pg_status pg_batch_destroy(pg_batch* plan);

#ifdef __cplusplus
}
#endif

#endif /* PATHGRAPH_H */
