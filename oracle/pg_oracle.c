/*
 * pg_oracle.c -- FP64 single-threaded oracle for path-graph rendering of
 * participating media (Hu, Deng, Luan, Hasan, Marschner: "Rendering
 * Participating Media Using Path Graphs", arXiv 2404.11894).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark call this code.  It shares nothing with the GPU
 * library (no headers, helpers or tables) and is written for a reader who
 * checks it against the paper, not for speed: plain loops in the order of the
 * method's own statement, double precision throughout.
 *
 * What it computes, step by step (paper sections in brackets):
 *   1. quantise positions to 20-bit integers per axis;
 *   2. neighbour sets N(i): i itself, then the K-1 nearest other vertices by
 *      (squared integer distance, index), K = min(k, N)   [Sec. "Path Graph
 *      Framework": vertices of a neighbourhood share incoming radiance];
 *   3. marginal densities and MIS-weighted edge weights of the indirect and
 *      direct aggregation operators   [Sec. "Path Graph Operators",
 *      eqs. indirect-weight, ag-indirect, ag-direct];
 *   4. the direct term (aggregated, and the plain path-traced one used for the
 *      final output)   [eq. ag-direct; "Handling direct Light" paragraph];
 *   5. the initial incoming indirect radiance, either the path tracer's own
 *      estimate or zero   ["Path graph solver" paragraph];
 *   6. D iterations of aggregation followed by propagation along continuation
 *      edges   [eqs. ag-mf, rte-pg, rte-mff];
 *   7. the output radiance of each path's first continuation edge, averaged
 *      into its pixel   ["Final output" paragraph];
 *   8. the reverse-mode derivative of an image-space objective with respect to
 *      the per-vertex albedo, a trilinear albedo grid and the HG parameter g
 *      (project addition, paths held fixed, sampling pdfs held fixed).
 *
 * Readings taken where the paper is silent (all stated again in the Python
 * wrapper and in the design notes):
 *   - neighbours are the k nearest (self first) instead of random clusters;
 *     the marginal density of a receiver sums over ITS neighbour set;
 *   - phase function: Henyey-Greenstein, cosine between travel directions;
 *     1 + g^2 - 2 g mu is evaluated as (1-g)^2 + 2 g u with u = |a-b|^2 / 2;
 *   - the sun is a delta light: no MIS, each neighbour's shadow-ray estimate
 *     is averaged with weight 1/K;
 *   - with delta tracking the propagation factor transmittance / free-flight
 *     pdf equals 1/sigma_t at the collision, which turns sigma_s * phase into
 *     albedo * phase; propagation therefore is a shift along the path;
 *   - more light types (the constant terms only): a point light is a delta
 *     light whose direction differs per vertex; like the sun it takes no MIS,
 *     each neighbour's shadow-ray sample (its direction and irradiance)
 *     counts with weight 1/K at the receiver, evaluated with the receiver's
 *     phase function, and the own direct term adds the vertex's own sample;
 *   - extra first-vertex samples (Sec. "Rendering System", handling direct
 *     light): with M > 0 extra emitter samples recorded at a path's first
 *     vertex, the pixel uses their emitter-sampling estimate
 *       d_fb = (1/M) sum_m ( rho(sun) Ls_m + rho(we_m) Le_m / p_e )
 *     in place of the non-aggregated direct term d_pt; the propagation keeps
 *     using the aggregated direct term.  Emitter sampling alone is unbiased
 *     for the sun and the environment, so the phase-sampled escape at v0
 *     (part of d_pt) is not added again;
 *   - volume emission (Sec. "Radiative Transfer Equation in a Medium"): the
 *     direct incoming radiance is Q + G L_v.  With delta tracking, G L_v
 *     along the segment from v to its successor u is estimated at the
 *     collision u by L_v(u) / sigma_t(u) =: e_u, an input per vertex
 *     (l_emit).  e_u is a phase-sampled direct sample at v, so it is
 *     aggregated with the same weights as the indirect sample arriving from
 *     u; adding e_u to the radiance leaving u toward its predecessor,
 *     y_u = e_u + alpha_u (d_agg_u + aggregated indirect), gives exactly
 *     that, and the pixel gets the e of the camera ray's first collision.
 *     The propagated vector L+ then holds the emission arriving from the
 *     successor plus the indirect radiance; with init zero it starts at the
 *     former (known before any iteration), so every iterate equals the one
 *     of the decomposition L = L^o + L^+ with the emission inside L^o.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_INPUT -4
#define OR_ERR_NOMEM -6

typedef struct or_scene {
    int64_t n_vertices, n_paths;
    int32_t width, height, spp, pad_;
    const int64_t* path_offsets;   /* [P+1] */
    const float* pos;              /* [N][3] */
    const float* dir_in;           /* [N][3] travel direction arriving at the vertex */
    const float* dir_out;          /* [N][3] phase-sampled continuation direction */
    const float* albedo;           /* [N] */
    const float* l_sun;            /* [N][3] */
    const float* dir_env;          /* [N][3] */
    const float* l_env;            /* [N][3] */
    const float* l_phase;          /* [N][3] */
    const float* e_cam;            /* [P][3] */
    const float* l_emit;           /* [N][3] or NULL: volume emission at the vertex */
    const uint32_t* cluster_key;   /* [N] uniform random keys (cluster neighbour relation) */
    const float* fb_l_sun;         /* [P][M][3] extra first-vertex samples, or NULL: sun x transmittance */
    const float* fb_dir_env;       /* [P][M][3] uniform-sphere environment directions */
    const float* fb_l_env;         /* [P][M][3] environment radiance x transmittance */
    int32_t n_extra;               /* M (0: no extra samples) */
    int32_t pad2_;
    const float* dir_pl;           /* [N][3] or NULL: unit direction toward a point light */
    const float* l_pl;             /* [N][3]: its intensity x shadow-ray transmittance / distance^2 */
} or_scene;

typedef struct or_params {
    int32_t k;            /* neighbours per vertex, self included */
    int32_t D;            /* propagation iterations */
    int32_t init;         /* 0: path-traced initial estimate, 1: zero */
    int32_t final_gather; /* 0: aggregate at the first vertex, 1: own sample only */
    int32_t neighbours;   /* 0: k nearest neighbours, 1: clusters (or_clusters) */
    int32_t pad_;
    double g;             /* HG parameter of the receiver's phase function */
    double g_s;           /* HG parameter of the sampling pdfs */
    double env_pdf;       /* solid-angle pdf of environment sampling (1/(4 pi)) */
    double sun_dir[3];    /* unit direction toward the sun */
} or_params;

/* Optional intermediate outputs of or_render (any pointer may be NULL). */
typedef struct or_trace {
    int64_t* row_ptr;  /* [N+1] rows of the neighbour lists (i*K for kNN) */
    int32_t* col;      /* [E] neighbour lists, E = row_ptr[N] */
    double* w_ind;     /* [E] indirect weights */
    double* w_ph;      /* [E] direct, phase-sampled weights */
    double* w_env;     /* [E] direct, emitter-sampled weights */
    double* d_agg;     /* [N][3] aggregated direct */
    double* b;         /* [N][3] albedo * aggregated direct */
    double* d_pt;      /* [N][3] path-traced direct */
    double* r;         /* [N] phase / pdf ratio of the own continuation */
    double* lplus0;    /* [N][3] initial incoming indirect radiance */
    double* lplus;     /* [N][3] after D iterations */
    double* traj;      /* [(D+1)][N][3] every iterate, t = 0..D */
    double* out_path;  /* [P][3] per-path output o_p (camera term excluded) */
} or_trace;

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------- phase function */

/* u = 1 - cos(angle) between unit vectors a and b, computed as |a - b|^2 / 2. */
static double one_minus_cos(const float* a, const float* b) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        double d = (double)a[c] - (double)b[c];
        s += d * d;
    }
    return 0.5 * s;
}
static double one_minus_cos_d(const float* a, const double* b) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        double d = (double)a[c] - b[c];
        s += d * d;
    }
    return 0.5 * s;
}

/* Henyey-Greenstein density as a function of u = 1 - cos(theta):
 *   HG_g = (1 - g^2) / (4 pi (1 + g^2 - 2 g cos)^(3/2)),  1 + g^2 - 2 g cos = (1-g)^2 + 2 g u. */
double or_hg(double g, double u) {
    double den = (1.0 - g) * (1.0 - g) + 2.0 * g * u;
    return (1.0 - g * g) / (4.0 * PI * den * sqrt(den));
}

/* d ln HG_g / d g at fixed u:  -2g/(1-g^2) - 3 (g - cos) / (1 + g^2 - 2 g cos). */
double or_hg_dlog(double g, double u) {
    double den = (1.0 - g) * (1.0 - g) + 2.0 * g * u;
    double mu = 1.0 - u;
    return -2.0 * g / (1.0 - g * g) - 3.0 * (g - mu) / den;
}

/* ---------------------------------------------------------- quantisation */

/* q = clamp(floor(x * 2^20), 0, 2^20 - 1) per axis.  Non-finite or outside
 * [0, 1] is an input error (the quantised value is still clamped). */
int or_quantize(int64_t n, const float* pos, int64_t* q) {
    int bad = 0;
    for (int64_t i = 0; i < n * 3; ++i) {
        double x = (double)pos[i];
        if (!(x >= 0.0 && x <= 1.0)) bad = 1;   /* also catches NaN */
        double s = floor(x * 1048576.0);
        if (!(s >= 0.0)) s = 0.0;
        if (s > 1048575.0) s = 1048575.0;
        q[i] = (int64_t)s;
    }
    return bad ? OR_ERR_INPUT : OR_OK;
}

/* ---------------------------------------------------------- neighbours */

static const int64_t* g_sort_q;   /* used only by the qsort comparator */
static int cmp_by_x(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    int64_t xa = g_sort_q[a * 3], xb = g_sort_q[b * 3];
    if (xa != xb) return xa < xb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int key_less(int64_t d1, int64_t j1, int64_t d2, int64_t j2) {
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

#define OR_KNN_SCAN_ROWS 512

/* The K-1 nearest j != i by (d2, j), by looking at every j: the definition
 * itself, O(n) per row.  Used when only a few rows are asked for, where
 * sorting all n vertices first would cost more than the rows. */
static void knn_row_scan(int64_t n, const int64_t* q, int64_t i, int64_t m, int64_t* bd, int64_t* bj) {
    int64_t filled = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        int64_t d2 = 0;
        for (int c = 0; c < 3; ++c) {
            int64_t dc = q[j * 3 + c] - q[i * 3 + c];
            d2 += dc * dc;
        }
        if (filled == m && (m == 0 || !key_less(d2, j, bd[m - 1], bj[m - 1]))) continue;
        int64_t p = filled < m ? filled : m - 1;
        while (p > 0 && key_less(d2, j, bd[p - 1], bj[p - 1])) {
            bd[p] = bd[p - 1];
            bj[p] = bj[p - 1];
            --p;
        }
        bd[p] = d2;
        bj[p] = j;
        if (filled < m) ++filled;
    }
}

/* Neighbour lists.  Row i: i first, then the K-1 nearest j != i ordered by
 * (squared distance of quantised positions, j), K = min(k, n).  rows == NULL
 * means every vertex (then nq must equal n).  Up to OR_KNN_SCAN_ROWS given
 * rows are answered by knn_row_scan.
 *
 * Search: vertices sorted by quantised x; from the query's place, walk left
 * and right, and stop in a direction once the x-gap alone exceeds the current
 * (K-1)-th distance -- every later vertex that way is farther still. */
int or_knn(int64_t n, const float* pos, int32_t k, int64_t nq, const int64_t* rows, int32_t* col) {
    if (n < 0 || k < 1 || nq < 0) return OR_ERR_ARG;
    if (n == 0) return OR_OK;
    int64_t K = k < n ? k : n;
    int64_t m = K - 1;
    if (rows && nq <= OR_KNN_SCAN_ROWS) {
        int64_t* q = (int64_t*)malloc((size_t)n * 3 * sizeof(int64_t));
        int64_t* bd = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
        int64_t* bj = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
        if (!q || !bd || !bj) {
            free(q); free(bd); free(bj);
            return OR_ERR_NOMEM;
        }
        int rc = or_quantize(n, pos, q);
        for (int64_t r = 0; r < nq; ++r) {
            knn_row_scan(n, q, rows[r], m, bd, bj);
            col[r * K] = (int32_t)rows[r];
            for (int64_t a = 0; a < m; ++a) col[r * K + 1 + a] = (int32_t)bj[a];
        }
        free(q); free(bd); free(bj);
        return rc;
    }
    int64_t* q = (int64_t*)malloc((size_t)n * 3 * sizeof(int64_t));
    int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* where = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* bd = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
    int64_t* bj = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!q || !order || !where || !bd || !bj) {
        free(q); free(order); free(where); free(bd); free(bj);
        return OR_ERR_NOMEM;
    }
    int rc = or_quantize(n, pos, q);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    g_sort_q = q;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_by_x);
    for (int64_t t = 0; t < n; ++t) where[order[t]] = t;

    for (int64_t r = 0; r < nq; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t filled = 0;
        for (int dir = -1; dir <= 1; dir += 2) {
            for (int64_t t = where[i] + dir; t >= 0 && t < n; t += dir) {
                int64_t j = order[t];
                int64_t dx = q[j * 3] - q[i * 3];
                if (filled == m && (m == 0 || dx * dx > bd[m - 1])) break;
                int64_t d2 = 0;
                for (int c = 0; c < 3; ++c) {
                    int64_t dc = q[j * 3 + c] - q[i * 3 + c];
                    d2 += dc * dc;
                }
                /* insert (d2, j) into the sorted list bd/bj of length filled <= m */
                if (filled == m && !key_less(d2, j, bd[m - 1], bj[m - 1])) continue;
                int64_t p = filled < m ? filled : m - 1;
                while (p > 0 && key_less(d2, j, bd[p - 1], bj[p - 1])) {
                    bd[p] = bd[p - 1];
                    bj[p] = bj[p - 1];
                    --p;
                }
                bd[p] = d2;
                bj[p] = j;
                if (filled < m) ++filled;
            }
        }
        col[r * K] = (int32_t)i;
        for (int64_t a = 0; a < m; ++a) col[r * K + 1 + a] = (int32_t)bj[a];
    }
    free(q); free(order); free(where); free(bd); free(bj);
    return rc;
}

/* ---------------------------------------------------------- clusters */

#define OR_CLUSTER_ROUNDS 4

static int64_t qdist2(const int64_t* q, int64_t a, int64_t b) {
    int64_t d2 = 0;
    for (int c = 0; c < 3; ++c) {
        int64_t d = q[a * 3 + c] - q[b * 3 + c];
        d2 += d * d;
    }
    return d2;
}

static const uint32_t* g_sort_key;   /* used only by the qsort comparators */
static const int32_t* g_sort_centre;
static int cmp_by_key(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    uint32_t ka = g_sort_key[a], kb = g_sort_key[b];
    if (ka != kb) return ka < kb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}
static int cmp_by_centre(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    int32_t ca = g_sort_centre[a], cb = g_sort_centre[b];
    if (ca != cb) return ca < cb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The paper's neighbour relation (Sec. "Path Graph Framework"; Sec.
 * "Rendering System", path graph solver): disjoint clusters around randomly
 * chosen centres, large clusters split again.  Readings:
 *   - the random choice is a uniform 32-bit key per vertex, an input; vertex
 *     i is a centre when key_i < floor(2^32 / K), so each vertex is one with
 *     probability 1/K and there are about N/K centres; the vertex with the
 *     smallest (key, id) always is one;
 *   - every vertex joins the nearest centre, nearest by (squared distance of
 *     the quantised positions, centre id);
 *   - a cluster is large when it has more than 2K members.  A large cluster
 *     of s members takes its ceil(s/K) members of smallest (key, id) as new
 *     centres and each of its members joins the nearest of those, as above.
 *     This repeats, for the clusters still large, up to OR_CLUSTER_ROUNDS
 *     rounds.
 * centre[i] receives the id of the centre of i's cluster. */
int or_clusters(int64_t n, const float* pos, const uint32_t* key, int32_t K, int32_t* centre) {
    if (n < 0 || K < 1 || (n > 0 && (!pos || !key || !centre))) return OR_ERR_ARG;
    if (n == 0) return OR_OK;
    int64_t* q = (int64_t*)malloc((size_t)n * 3 * sizeof(int64_t));
    int64_t* ctr = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* mem = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!q || !ctr || !order || !mem) {
        free(q); free(ctr); free(order); free(mem);
        return OR_ERR_NOMEM;
    }
    int rc = or_quantize(n, pos, q);
    const uint64_t thr = ((uint64_t)1 << 32) / (uint64_t)K;
    int64_t first = 0;
    for (int64_t i = 1; i < n; ++i)
        if (key[i] < key[first]) first = i;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if ((uint64_t)key[i] < thr || i == first) ctr[m++] = i;
    for (int64_t i = 0; i < n; ++i) {
        int64_t best = -1, bd = 0;
        for (int64_t c = 0; c < m; ++c) {
            int64_t d2 = qdist2(q, i, ctr[c]);
            if (best < 0 || key_less(d2, ctr[c], bd, best)) {
                bd = d2;
                best = ctr[c];
            }
        }
        centre[i] = (int32_t)best;
    }
    for (int round = 0; round < OR_CLUSTER_ROUNDS; ++round) {
        /* group by centre: order[] lists the vertices by (centre, id) */
        for (int64_t i = 0; i < n; ++i) order[i] = i;
        g_sort_centre = centre;
        qsort(order, (size_t)n, sizeof(int64_t), cmp_by_centre);
        int split = 0;
        for (int64_t a = 0; a < n;) {
            int64_t e = a;
            while (e < n && centre[order[e]] == centre[order[a]]) ++e;
            int64_t sz = e - a;
            if (sz > 2 * (int64_t)K) {
                split = 1;
                for (int64_t t = 0; t < sz; ++t) mem[t] = order[a + t];
                g_sort_key = key;
                qsort(mem, (size_t)sz, sizeof(int64_t), cmp_by_key);
                int64_t nc = (sz + K - 1) / K;
                /* mem[0..nc) are the new centres; assign every member */
                for (int64_t t = 0; t < sz; ++t) {
                    int64_t i = mem[t], best = -1, bd = 0;
                    for (int64_t c = 0; c < nc; ++c) {
                        int64_t d2 = qdist2(q, i, mem[c]);
                        if (best < 0 || key_less(d2, mem[c], bd, best)) {
                            bd = d2;
                            best = mem[c];
                        }
                    }
                    centre[i] = (int32_t)best;
                }
            }
            a = e;
        }
        if (!split) break;
    }
    free(q); free(ctr); free(order); free(mem);
    return rc;
}

/* ---------------------------------------------------------- edge weights */

/* Per receiver i with neighbour list nb[0..K-1] (nb[0] == i):
 *   M+_ij = sum_l p_l(w_j)                  marginal of the continuation sample of j
 *   Mp_ij = M+_ij + K p_e                   same sample as a direct-light sample
 *   Me_ij = sum_l p_l(we_j) + K p_e         marginal of j's emitter sample
 *   w+_ij = rho_i(w_j) / M+_ij,  wp_ij = rho_i(w_j) / Mp_ij,  we_ij = rho_i(we_j) / Me_ij
 *   d_agg_i = rho_i(sun) (1/K) sum_j Ls_j + sum_j (we_ij Le_j + wp_ij Lp_j)
 * with p_l = HG_{g_s} about l's arriving direction and rho_i = HG_g about i's.
 * (eqs. indirect-weight, ag-indirect and ag-direct; sun handled as a delta light.) */
static void receiver_weights(const or_scene* s, const or_params* p, int64_t i, const int32_t* nb,
                             int64_t K, double* wi, double* wp, double* we, double dagg[3]) {
    const float* ti = s->dir_in + i * 3;
    double Kpe = (double)K * p->env_pdf;
    double sum_ls[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 3; ++c) dagg[c] = 0.0;
    for (int64_t a = 0; a < K; ++a) {
        int64_t j = nb[a];
        const float* wj = s->dir_out + j * 3;
        const float* ej = s->dir_env + j * 3;
        double mplus = 0.0, menv = 0.0;
        for (int64_t b = 0; b < K; ++b) {
            const float* tl = s->dir_in + (int64_t)nb[b] * 3;
            mplus += or_hg(p->g_s, one_minus_cos(tl, wj));
            menv += or_hg(p->g_s, one_minus_cos(tl, ej));
        }
        menv += Kpe;
        double rho = or_hg(p->g, one_minus_cos(ti, wj));
        double rho_e = or_hg(p->g, one_minus_cos(ti, ej));
        wi[a] = rho / mplus;
        wp[a] = rho / (mplus + Kpe);
        we[a] = rho_e / menv;
        for (int c = 0; c < 3; ++c) {
            sum_ls[c] += s->l_sun[j * 3 + c];
            dagg[c] += we[a] * s->l_env[j * 3 + c] + wp[a] * s->l_phase[j * 3 + c];
        }
    }
    double rho_sun = or_hg(p->g, one_minus_cos_d(ti, p->sun_dir));
    for (int c = 0; c < 3; ++c) dagg[c] += rho_sun * sum_ls[c] / (double)K;
    if (s->dir_pl && s->l_pl) {   /* point light: delta, weight 1/K per neighbour sample */
        for (int64_t a = 0; a < K; ++a) {
            int64_t j = nb[a];
            double rho_pl = or_hg(p->g, one_minus_cos(ti, s->dir_pl + j * 3));
            for (int c = 0; c < 3; ++c) dagg[c] += rho_pl * s->l_pl[j * 3 + c] / (double)K;
        }
    }
}

/* Plain path-traced direct term of vertex i (one sun sample, one environment
 * sample and the phase sample combined by the balance heuristic) and the
 * phase / pdf ratio of its own continuation. */
static void own_direct(const or_scene* s, const or_params* p, int64_t i, double dpt[3], double* r) {
    const float* ti = s->dir_in + i * 3;
    double u_sun = one_minus_cos_d(ti, p->sun_dir);
    double u_env = one_minus_cos(ti, s->dir_env + i * 3);
    double u_out = one_minus_cos(ti, s->dir_out + i * 3);
    double f_sun = or_hg(p->g, u_sun);
    double f_env = or_hg(p->g, u_env) / (or_hg(p->g_s, u_env) + p->env_pdf);
    double f_out = or_hg(p->g, u_out) / (or_hg(p->g_s, u_out) + p->env_pdf);
    for (int c = 0; c < 3; ++c)
        dpt[c] = f_sun * s->l_sun[i * 3 + c] + f_env * s->l_env[i * 3 + c] + f_out * s->l_phase[i * 3 + c];
    if (s->dir_pl && s->l_pl) {
        double f_pl = or_hg(p->g, one_minus_cos(ti, s->dir_pl + i * 3));
        for (int c = 0; c < 3; ++c) dpt[c] += f_pl * s->l_pl[i * 3 + c];
    }
    *r = or_hg(p->g, u_out) / or_hg(p->g_s, u_out);
}

/* Edge weights and direct terms for a set of receivers (rows == NULL: all).
 * col holds the receivers' neighbour lists, K entries each, in row order. */
int or_edges(const or_scene* s, const or_params* p, int32_t K, int64_t nq, const int64_t* rows,
             const int32_t* col, double* w_ind, double* w_ph, double* w_env, double* d_agg,
             double* d_pt, double* r) {
    if (K < 1) return OR_ERR_ARG;
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = rows ? rows[q] : q;
        receiver_weights(s, p, i, col + q * K, K, w_ind + q * K, w_ph + q * K, w_env + q * K, d_agg + q * 3);
        own_direct(s, p, i, d_pt + q * 3, r + q);
    }
    return OR_OK;
}

/* ---------------------------------------------------------- trilinear albedo */

/* alpha_i = trilinear interpolation of a cell-centred R^3 grid ([z][y][x]).
 * Per axis u = R x - 0.5, i0 = floor(u), f = u - i0, corner indices i0 and i0+1
 * each clamped to [0, R-1], weights 1-f and f. */
static void trilerp_corners(int32_t R, const float* x, int64_t idx[8], double w[8]) {
    int64_t i0[3], i1[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double u = (double)R * (double)x[a] - 0.5;
        double fl = floor(u);
        f[a] = u - fl;
        int64_t lo = (int64_t)fl, hi = lo + 1;
        i0[a] = lo < 0 ? 0 : (lo > R - 1 ? R - 1 : lo);
        i1[a] = hi < 0 ? 0 : (hi > R - 1 ? R - 1 : hi);
    }
    for (int c = 0; c < 8; ++c) {
        int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        int64_t ix = bx ? i1[0] : i0[0], iy = by ? i1[1] : i0[1], iz = bz ? i1[2] : i0[2];
        idx[c] = (iz * R + iy) * R + ix;
        w[c] = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
    }
}

int or_albedo_from_grid(int64_t n, const float* pos, int32_t R, const float* grid, double* alpha) {
    if (R < 1) return OR_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) {
        int64_t idx[8];
        double w[8];
        trilerp_corners(R, pos + i * 3, idx, w);
        double a = 0.0;
        for (int c = 0; c < 8; ++c) a += w[c] * (double)grid[idx[c]];
        alpha[i] = a;
    }
    return OR_OK;
}

/* ---------------------------------------------------------- forward render */

/* Direct term of the pixel of path q with first vertex v0: the extra
 * emitter samples' estimate when there are any, else d_pt (set by the
 * caller).  With dg != NULL also its derivative with respect to g. */
static void first_direct(const or_scene* s, const or_params* p, int64_t q, int64_t v0, double d[3], double dg[3]) {
    const float* ti = s->dir_in + v0 * 3;
    const int64_t M = s->n_extra;
    double u_sun = one_minus_cos_d(ti, p->sun_dir);
    double rs = or_hg(p->g, u_sun), hs = or_hg_dlog(p->g, u_sun);
    for (int c = 0; c < 3; ++c) {
        d[c] = 0.0;
        if (dg) dg[c] = 0.0;
    }
    for (int64_t m = 0; m < M; ++m) {
        const size_t o = ((size_t)q * M + m) * 3;
        double u = one_minus_cos(ti, s->fb_dir_env + o);
        double re = or_hg(p->g, u), he = or_hg_dlog(p->g, u);
        for (int c = 0; c < 3; ++c) {
            d[c] += (rs * s->fb_l_sun[o + c] + re * s->fb_l_env[o + c] / p->env_pdf) / (double)M;
            if (dg) dg[c] += (rs * hs * s->fb_l_sun[o + c] + re * he * s->fb_l_env[o + c] / p->env_pdf) / (double)M;
        }
    }
    if (s->dir_pl && s->l_pl) {   /* a point light keeps the vertex's own sample */
        double u = one_minus_cos(ti, s->dir_pl + v0 * 3);
        double rp = or_hg(p->g, u), hp = or_hg_dlog(p->g, u);
        for (int c = 0; c < 3; ++c) {
            d[c] += rp * s->l_pl[v0 * 3 + c];
            if (dg) dg[c] += rp * hp * s->l_pl[v0 * 3 + c];
        }
    }
}

static int has_extra(const or_scene* s) {
    return s->n_extra > 0 && s->fb_l_sun && s->fb_dir_env && s->fb_l_env;
}

/* Volume emission leaving vertex i toward its predecessor, channel c. */
static double emit(const or_scene* s, int64_t i, int c) {
    return s->l_emit ? (double)s->l_emit[i * 3 + c] : 0.0;
}

typedef struct {
    int64_t N, P, K, E;
    int keep;       /* 1: traj holds every iterate t = 0..D; 0: three rotating slots */
    int64_t* rp;    /* [N+1] row i = edges rp[i] .. rp[i+1]-1 */
    int32_t* col;
    double *wi, *wp, *we, *dagg, *b, *dpt, *r, *alpha;
    double* traj;   /* (D+1) * N * 3 when keep, else 3 * N * 3 */
} fwd_state;

/* iterate t inside the state's storage */
static double* iterate(const fwd_state* f, int t, int D) {
    (void)D;
    size_t slot = f->keep ? (size_t)t : (t == 0 ? 0u : (size_t)(1 + (t & 1)));
    return f->traj + slot * (size_t)f->N * 3;
}

static void free_state(fwd_state* f) {
    free(f->rp); free(f->col); free(f->wi); free(f->wp); free(f->we); free(f->dagg); free(f->b);
    free(f->dpt); free(f->r); free(f->alpha); free(f->traj);
    memset(f, 0, sizeof(*f));
}

static int validate(const or_scene* s, const or_params* p) {
    if (!s || !p || s->n_vertices < 0 || s->n_paths < 0 || p->k < 1 || p->D < 0) return OR_ERR_ARG;
    if (s->width < 1 || s->height < 1 || s->spp < 1) return OR_ERR_ARG;
    if ((int64_t)s->width * s->height * s->spp != s->n_paths) return OR_ERR_ARG;
    if (!(fabs(p->g) < 1.0) || !(fabs(p->g_s) < 1.0) || !(p->env_pdf > 0.0)) return OR_ERR_ARG;
    if (p->neighbours != 0 && p->neighbours != 1) return OR_ERR_ARG;
    if (p->neighbours == 1 && s->n_vertices > 0 && !s->cluster_key) return OR_ERR_ARG;
    if (s->n_extra < 0) return OR_ERR_ARG;
    if (s->path_offsets[0] != 0 || s->path_offsets[s->n_paths] != s->n_vertices) return OR_ERR_ARG;
    for (int64_t q = 0; q < s->n_paths; ++q)
        if (s->path_offsets[q + 1] < s->path_offsets[q]) return OR_ERR_ARG;
    return OR_OK;
}

/* Runs steps 1-7.  alpha_override (N doubles) replaces the scene albedo when
 * not NULL.  Fills the forward state (every iterate kept) and the image. */
static int forward(const or_scene* s, const or_params* p, const double* alpha_override, int keep,
                   fwd_state* f, double* image, double* out_path) {
    int rc = validate(s, p);
    if (rc) return rc;
    const int64_t N = s->n_vertices, P = s->n_paths;
    const int64_t K = N == 0 ? 0 : (p->k < N ? p->k : N);
    const int D = p->D;
    memset(f, 0, sizeof(*f));
    f->N = N; f->P = P; f->K = K; f->keep = keep;
    size_t n3 = (size_t)(N > 0 ? N * 3 : 1);

    /* steps 1-2: neighbour sets as rows of a CSR (row i: i's neighbours) */
    f->rp = (int64_t*)malloc((size_t)(N + 1) * sizeof(int64_t));
    if (!f->rp) { free_state(f); return OR_ERR_NOMEM; }
    f->rp[0] = 0;
    if (p->neighbours == 0) {
        for (int64_t i = 0; i < N; ++i) f->rp[i + 1] = (i + 1) * K;
        f->col = (int32_t*)malloc((size_t)(N * K > 0 ? N * K : 1) * sizeof(int32_t));
        if (!f->col) { free_state(f); return OR_ERR_NOMEM; }
        if (N > 0 && (rc = or_knn(N, s->pos, p->k, N, NULL, f->col))) { free_state(f); return rc; }
    } else {
        /* clusters: row i lists the members of i's cluster, ids ascending */
        int32_t* ctr = (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
        int64_t* order = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
        int64_t* size = (int64_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
        int64_t* first = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
        if (!ctr || !order || !size || !first) {
            free(ctr); free(order); free(size); free(first); free_state(f);
            return OR_ERR_NOMEM;
        }
        rc = or_clusters(N, s->pos, s->cluster_key, p->k, ctr);
        if (rc) { free(ctr); free(order); free(size); free(first); free_state(f); return rc; }
        for (int64_t i = 0; i < N; ++i) order[i] = i;
        g_sort_centre = ctr;
        qsort(order, (size_t)N, sizeof(int64_t), cmp_by_centre);
        for (int64_t i = 0; i < N; ++i) ++size[ctr[i]];
        for (int64_t t = N - 1; t >= 0; --t) first[ctr[order[t]]] = t;   /* members start in order[] */
        for (int64_t i = 0; i < N; ++i) f->rp[i + 1] = f->rp[i] + size[ctr[i]];
        f->col = (int32_t*)malloc((size_t)(f->rp[N] > 0 ? f->rp[N] : 1) * sizeof(int32_t));
        if (!f->col) { free(ctr); free(order); free(size); free(first); free_state(f); return OR_ERR_NOMEM; }
        for (int64_t i = 0; i < N; ++i)
            for (int64_t a = 0; a < size[ctr[i]]; ++a) f->col[f->rp[i] + a] = (int32_t)order[first[ctr[i]] + a];
        free(ctr); free(order); free(size); free(first);
    }
    f->E = f->rp[N];
    size_t nE = (size_t)(f->E > 0 ? f->E : 1);
    f->wi = (double*)malloc(nE * sizeof(double));
    f->wp = (double*)malloc(nE * sizeof(double));
    f->we = (double*)malloc(nE * sizeof(double));
    f->dagg = (double*)malloc(n3 * sizeof(double));
    f->b = (double*)malloc(n3 * sizeof(double));
    f->dpt = (double*)malloc(n3 * sizeof(double));
    f->r = (double*)malloc((N > 0 ? N : 1) * sizeof(double));
    f->alpha = (double*)malloc((N > 0 ? N : 1) * sizeof(double));
    f->traj = (double*)calloc((size_t)(keep ? D + 1 : 3) * n3, sizeof(double));
    if (!f->wi || !f->wp || !f->we || !f->dagg || !f->b || !f->dpt || !f->r || !f->alpha || !f->traj) {
        free_state(f);
        return OR_ERR_NOMEM;
    }
    for (int64_t i = 0; i < N; ++i) f->alpha[i] = alpha_override ? alpha_override[i] : (double)s->albedo[i];

    /* steps 3-4: weights, direct terms, b = alpha * d_agg */
    for (int64_t i = 0; i < N; ++i) {
        const int64_t e0 = f->rp[i], ki = f->rp[i + 1] - e0;
        receiver_weights(s, p, i, f->col + e0, ki, f->wi + e0, f->wp + e0, f->we + e0, f->dagg + i * 3);
        own_direct(s, p, i, f->dpt + i * 3, f->r + i);
        for (int c = 0; c < 3; ++c)
            f->b[i * 3 + c] = emit(s, i, c) + f->alpha[i] * f->dagg[i * 3 + c];
    }
    /* step 5: initial L+_0 (traj[0]), the radiance arriving at v from its
     * successor u along the continuation (the last vertex of a path has none):
     *   init PT:   the path tracer's estimate e_u + alpha_u (d_pt_u + r_u L+_0(u));
     *   init zero: the unknown indirect part starts at 0, which leaves e_u, the
     *              emission collected at u (part of the known direct radiance). */
    double* L0 = f->traj;
    for (int64_t q = 0; q < P; ++q) {
        int64_t a = s->path_offsets[q], e = s->path_offsets[q + 1];
        for (int64_t v = e - 2; v >= a; --v) {
            int64_t u = v + 1;
            for (int c = 0; c < 3; ++c)
                L0[v * 3 + c] = p->init == 0
                    ? emit(s, u, c) + f->alpha[u] * (f->dpt[u * 3 + c] + f->r[u] * L0[u * 3 + c])
                    : emit(s, u, c);
        }
    }
    /* step 6: D iterations.  Aggregation at every vertex i:
     *   y_i = b_i + alpha_i sum_j w+_ij L+(j)      (b_i = e_i + alpha_i d_agg_i)
     * then propagation: L+(v) = y(succ v), 0 at a path's last vertex. */
    double* y = (double*)malloc(n3 * sizeof(double));
    if (!y) { free_state(f); return OR_ERR_NOMEM; }
    for (int t = 1; t <= D; ++t) {
        const double* Lp = iterate(f, t - 1, D);
        double* Ln = iterate(f, t, D);
        for (int64_t i = 0; i < N; ++i) {
            double z[3] = {0.0, 0.0, 0.0};
            for (int64_t a = f->rp[i]; a < f->rp[i + 1]; ++a) {
                int64_t j = f->col[a];
                for (int c = 0; c < 3; ++c) z[c] += f->wi[a] * Lp[j * 3 + c];
            }
            for (int c = 0; c < 3; ++c) y[i * 3 + c] = f->b[i * 3 + c] + f->alpha[i] * z[c];
        }
        for (int64_t q = 0; q < P; ++q) {
            int64_t a = s->path_offsets[q], e = s->path_offsets[q + 1];
            for (int64_t v = a; v < e; ++v)
                for (int c = 0; c < 3; ++c) Ln[v * 3 + c] = (v + 1 < e) ? y[(v + 1) * 3 + c] : 0.0;
        }
    }
    free(y);
    /* step 7: output of each path's first continuation edge, then pixels.
     * o_p = e_v0 + alpha_v0 (d_pt_v0 + sum_j w+_v0j L+_D(j))   (final_gather == 0)
     * o_p = e_v0 + alpha_v0 (d_pt_v0 + r_v0 L+_D(v0))          (final_gather == 1)
     * (d_fb of the extra first-vertex samples in place of d_pt_v0 when given) */
    const double* LD = iterate(f, D, D);
    const int64_t npix = (int64_t)s->width * s->height;
    for (int64_t px = 0; px < npix * 3; ++px) image[px] = 0.0;
    for (int64_t q = 0; q < P; ++q) {
        double o[3] = {0.0, 0.0, 0.0};
        int64_t v0 = s->path_offsets[q];
        if (s->path_offsets[q + 1] > v0) {
            double in[3] = {0.0, 0.0, 0.0};
            if (p->final_gather == 0) {
                for (int64_t a = f->rp[v0]; a < f->rp[v0 + 1]; ++a) {
                    int64_t j = f->col[a];
                    for (int c = 0; c < 3; ++c) in[c] += f->wi[a] * LD[j * 3 + c];
                }
            } else {
                for (int c = 0; c < 3; ++c) in[c] = f->r[v0] * LD[v0 * 3 + c];
            }
            double dd[3] = {f->dpt[v0 * 3], f->dpt[v0 * 3 + 1], f->dpt[v0 * 3 + 2]};
            if (has_extra(s)) first_direct(s, p, q, v0, dd, NULL);
            for (int c = 0; c < 3; ++c) o[c] = emit(s, v0, c) + f->alpha[v0] * (dd[c] + in[c]);
        }
        if (out_path)
            for (int c = 0; c < 3; ++c) out_path[q * 3 + c] = o[c];
        int64_t px = q / s->spp;
        for (int c = 0; c < 3; ++c) image[px * 3 + c] += ((double)s->e_cam[q * 3 + c] + o[c]) / (double)s->spp;
    }
    return OR_OK;
}

/* Forward render in FP64.  image: [H][W][3].  alpha_override: [N] or NULL. */
int or_render(const or_scene* s, const or_params* p, const double* alpha_override, double* image,
              or_trace* tr) {
    fwd_state f;
    int rc = forward(s, p, alpha_override, tr && tr->traj ? 1 : 0, &f, image, tr ? tr->out_path : NULL);
    if (rc) return rc;
    if (tr) {
        const int64_t N = f.N, E = f.E;
        if (tr->row_ptr) memcpy(tr->row_ptr, f.rp, (size_t)(N + 1) * sizeof(int64_t));
        if (tr->col) memcpy(tr->col, f.col, (size_t)E * sizeof(int32_t));
        if (tr->w_ind) memcpy(tr->w_ind, f.wi, (size_t)E * sizeof(double));
        if (tr->w_ph) memcpy(tr->w_ph, f.wp, (size_t)E * sizeof(double));
        if (tr->w_env) memcpy(tr->w_env, f.we, (size_t)E * sizeof(double));
        if (tr->d_agg) memcpy(tr->d_agg, f.dagg, (size_t)(N * 3) * sizeof(double));
        if (tr->b) memcpy(tr->b, f.b, (size_t)(N * 3) * sizeof(double));
        if (tr->d_pt) memcpy(tr->d_pt, f.dpt, (size_t)(N * 3) * sizeof(double));
        if (tr->r) memcpy(tr->r, f.r, (size_t)N * sizeof(double));
        if (tr->lplus0) memcpy(tr->lplus0, f.traj, (size_t)(N * 3) * sizeof(double));
        if (tr->lplus) memcpy(tr->lplus, iterate(&f, p->D, p->D), (size_t)(N * 3) * sizeof(double));
        if (tr->traj) memcpy(tr->traj, f.traj, (size_t)(p->D + 1) * N * 3 * sizeof(double));
    }
    free_state(&f);
    return OR_OK;
}

/* ---------------------------------------------------------- reverse mode */

/* Gradient of  sum_px <grad_image[px], I[px]>  with respect to
 *   - the per-vertex albedo (grad_alpha, [N]),
 *   - the albedo grid (grad_grid, [R^3]) when grid != NULL, in which case the
 *     albedo is the trilinear interpolation of the grid (the scene albedo is
 *     then ignored),
 *   - the receiver-side HG parameter g (grad_g), with the sampling pdfs (g_s)
 *     and the paths held fixed.
 * Every step reverses a step of the forward pass, in the opposite order. */
int or_backward(const or_scene* s, const or_params* p, int32_t R, const float* grid,
                const double* grad_image, double* grad_alpha, double* grad_grid, double* grad_g,
                double* image) {
    const int64_t N = s->n_vertices;
    double* alpha = NULL;
    if (grid) {
        if (R < 1) return OR_ERR_ARG;
        alpha = (double*)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
        if (!alpha) return OR_ERR_NOMEM;
        or_albedo_from_grid(N, s->pos, R, grid, alpha);
    }
    fwd_state f;
    int rc = forward(s, p, alpha, 1, &f, image, NULL);
    if (rc) { free(alpha); return rc; }
    const int64_t P = s->n_paths;
    const int64_t* rp = f.rp;
    const int D = p->D;
    size_t n3 = (size_t)(N > 0 ? N * 3 : 1);
    double* abar = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double* dptbar = (double*)calloc(n3, sizeof(double));
    double* rbar = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double* bbar = (double*)calloc(n3, sizeof(double));
    double* lam = (double*)calloc(n3, sizeof(double));     /* adjoint of L+_t */
    double* lam2 = (double*)calloc(n3, sizeof(double));
    double* wbar = (double*)calloc((size_t)(f.E > 0 ? f.E : 1), sizeof(double));
    if (!abar || !dptbar || !rbar || !bbar || !lam || !lam2 || !wbar) {
        free(abar); free(dptbar); free(rbar); free(bbar); free(lam); free(lam2); free(wbar);
        free_state(&f); free(alpha);
        return OR_ERR_NOMEM;
    }
    const double* LD = f.traj + (size_t)D * N * 3;
    double gfb = 0.0;   /* d/dg through the extra first-vertex samples */

    /* reverse of step 7 */
    for (int64_t q = 0; q < P; ++q) {
        int64_t v0 = s->path_offsets[q];
        if (s->path_offsets[q + 1] <= v0) continue;
        int64_t px = q / s->spp;
        double ob[3];
        for (int c = 0; c < 3; ++c) ob[c] = grad_image[px * 3 + c] / (double)s->spp;
        double in[3] = {0.0, 0.0, 0.0};
        if (p->final_gather == 0) {
            for (int64_t a = rp[v0]; a < rp[v0 + 1]; ++a) {
                int64_t j = f.col[a];
                for (int c = 0; c < 3; ++c) in[c] += f.wi[a] * LD[j * 3 + c];
            }
        } else {
            for (int c = 0; c < 3; ++c) in[c] = f.r[v0] * LD[v0 * 3 + c];
        }
        if (has_extra(s)) {
            double dd[3], ddg[3];
            first_direct(s, p, q, v0, dd, ddg);
            for (int c = 0; c < 3; ++c) {
                abar[v0] += ob[c] * (dd[c] + in[c]);
                gfb += f.alpha[v0] * ob[c] * ddg[c];
            }
        } else {
            for (int c = 0; c < 3; ++c) {
                abar[v0] += ob[c] * (f.dpt[v0 * 3 + c] + in[c]);
                dptbar[v0 * 3 + c] += f.alpha[v0] * ob[c];
            }
        }
        if (p->final_gather == 0) {
            for (int64_t a = rp[v0]; a < rp[v0 + 1]; ++a) {
                int64_t j = f.col[a];
                for (int c = 0; c < 3; ++c) {
                    double zb = f.alpha[v0] * ob[c];
                    lam[j * 3 + c] += f.wi[a] * zb;
                    wbar[a] += zb * LD[j * 3 + c];
                }
            }
        } else {
            for (int c = 0; c < 3; ++c) {
                rbar[v0] += f.alpha[v0] * ob[c] * LD[v0 * 3 + c];
                lam[v0 * 3 + c] += f.alpha[v0] * f.r[v0] * ob[c];
            }
        }
    }
    /* reverse of step 6, t = D .. 1.  lam holds the adjoint of L+_t. */
    double* ybar = (double*)malloc(n3 * sizeof(double));
    if (!ybar) rc = OR_ERR_NOMEM;
    for (int t = D; t >= 1 && !rc; --t) {
        const double* Lp = f.traj + (size_t)(t - 1) * N * 3;
        /* propagation: L+_t(v) = y(v+1) inside a path */
        for (size_t e = 0; e < n3; ++e) ybar[e] = 0.0;
        for (int64_t q = 0; q < P; ++q) {
            int64_t a = s->path_offsets[q], e = s->path_offsets[q + 1];
            for (int64_t v = a; v + 1 < e; ++v)
                for (int c = 0; c < 3; ++c) ybar[(v + 1) * 3 + c] += lam[v * 3 + c];
        }
        /* aggregation: y_i = b_i + alpha_i z_i, z_i = sum_j w+_ij L+_{t-1}(j) */
        for (size_t e = 0; e < n3; ++e) lam2[e] = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double z[3] = {0.0, 0.0, 0.0};
            for (int64_t a = rp[i]; a < rp[i + 1]; ++a) {
                int64_t j = f.col[a];
                for (int c = 0; c < 3; ++c) z[c] += f.wi[a] * Lp[j * 3 + c];
            }
            for (int c = 0; c < 3; ++c) {
                bbar[i * 3 + c] += ybar[i * 3 + c];
                abar[i] += ybar[i * 3 + c] * z[c];
            }
            for (int64_t a = rp[i]; a < rp[i + 1]; ++a) {
                int64_t j = f.col[a];
                for (int c = 0; c < 3; ++c) {
                    double zb = f.alpha[i] * ybar[i * 3 + c];
                    lam2[j * 3 + c] += f.wi[a] * zb;
                    wbar[a] += zb * Lp[j * 3 + c];
                }
            }
        }
        double* tmp = lam; lam = lam2; lam2 = tmp;
    }
    free(ybar);
    /* reverse of step 5 (path-traced initial estimate), first vertex to last */
    if (!rc && p->init == 0) {
        const double* L0 = f.traj;
        for (int64_t q = 0; q < P; ++q) {
            int64_t a = s->path_offsets[q], e = s->path_offsets[q + 1];
            for (int64_t v = a; v + 1 < e; ++v) {
                int64_t u = v + 1;
                for (int c = 0; c < 3; ++c) {
                    double lb = lam[v * 3 + c];
                    abar[u] += lb * (f.dpt[u * 3 + c] + f.r[u] * L0[u * 3 + c]);
                    dptbar[u * 3 + c] += f.alpha[u] * lb;
                    rbar[u] += f.alpha[u] * lb * L0[u * 3 + c];
                    lam[u * 3 + c] += f.alpha[u] * f.r[u] * lb;
                }
            }
        }
    }
    /* reverse of step 4 and of the weights' dependence on g */
    double gg = gfb;
    for (int64_t i = 0; i < N && !rc; ++i) {
        const float* ti = s->dir_in + i * 3;
        double daggbar[3];
        for (int c = 0; c < 3; ++c) {
            abar[i] += bbar[i * 3 + c] * f.dagg[i * 3 + c];
            daggbar[c] = f.alpha[i] * bbar[i * 3 + c];
        }
        /* d/dg of rho_i(w) is rho_i(w) h(u); pdfs do not depend on g */
        double sum_ls[3] = {0.0, 0.0, 0.0};
        for (int64_t a = rp[i]; a < rp[i + 1]; ++a) {
            int64_t j = f.col[a];
            double h_out = or_hg_dlog(p->g, one_minus_cos(ti, s->dir_out + j * 3));
            double h_env = or_hg_dlog(p->g, one_minus_cos(ti, s->dir_env + j * 3));
            gg += wbar[a] * f.wi[a] * h_out;
            for (int c = 0; c < 3; ++c) {
                gg += daggbar[c] * (f.we[a] * h_env * s->l_env[j * 3 + c] +
                                    f.wp[a] * h_out * s->l_phase[j * 3 + c]);
                sum_ls[c] += s->l_sun[j * 3 + c];
            }
        }
        double u_sun = one_minus_cos_d(ti, p->sun_dir);
        double rho_sun = or_hg(p->g, u_sun), h_sun = or_hg_dlog(p->g, u_sun);
        for (int c = 0; c < 3; ++c) gg += daggbar[c] * rho_sun * h_sun * sum_ls[c] / (double)(rp[i + 1] - rp[i]);
        if (s->dir_pl && s->l_pl) {
            for (int64_t a = rp[i]; a < rp[i + 1]; ++a) {
                int64_t j = f.col[a];
                double u = one_minus_cos(ti, s->dir_pl + j * 3);
                double w = or_hg(p->g, u) * or_hg_dlog(p->g, u) / (double)(rp[i + 1] - rp[i]);
                for (int c = 0; c < 3; ++c) gg += daggbar[c] * w * s->l_pl[j * 3 + c];
            }
            double u = one_minus_cos(ti, s->dir_pl + i * 3);
            double w = or_hg(p->g, u) * or_hg_dlog(p->g, u);
            for (int c = 0; c < 3; ++c) gg += dptbar[i * 3 + c] * w * s->l_pl[i * 3 + c];
        }
        /* own direct term and continuation ratio */
        double u_env = one_minus_cos(ti, s->dir_env + i * 3);
        double u_out = one_minus_cos(ti, s->dir_out + i * 3);
        double f_env = or_hg(p->g, u_env) / (or_hg(p->g_s, u_env) + p->env_pdf);
        double f_out = or_hg(p->g, u_out) / (or_hg(p->g_s, u_out) + p->env_pdf);
        double h_env = or_hg_dlog(p->g, u_env), h_out = or_hg_dlog(p->g, u_out);
        for (int c = 0; c < 3; ++c)
            gg += dptbar[i * 3 + c] * (rho_sun * h_sun * s->l_sun[i * 3 + c] + f_env * h_env * s->l_env[i * 3 + c] +
                                       f_out * h_out * s->l_phase[i * 3 + c]);
        gg += rbar[i] * f.r[i] * h_out;
    }
    if (!rc) {
        if (grad_g) *grad_g = gg;
        if (grad_alpha) memcpy(grad_alpha, abar, (size_t)N * sizeof(double));
        if (grad_grid && grid) {
            for (int64_t e = 0; e < (int64_t)R * R * R; ++e) grad_grid[e] = 0.0;
            for (int64_t i = 0; i < N; ++i) {
                int64_t idx[8];
                double w[8];
                trilerp_corners(R, s->pos + i * 3, idx, w);
                for (int c = 0; c < 8; ++c) grad_grid[idx[c]] += abar[i] * w[c];
            }
        }
    }
    free(abar); free(dptbar); free(rbar); free(bbar); free(lam); free(lam2); free(wbar);
    free_state(&f); free(alpha);
    return rc;
}
