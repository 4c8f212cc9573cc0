// pg_render.hip -- the forward pipeline in the internal, spatially sorted
// layout: grid build and kNN, aggregation operators, per-path pass, D
// iterations of aggregation + propagation, output to pixels.  Host code.
#include "pg_api_common.h"

namespace pg {

int resolve_schedule(const pg_params* q) { return q->schedule ? q->schedule : PG_SCHED_TWO_PASS; }

void carve_render(Carver& cv, RenderBufs& r, const pg_paths* p, const pg_params* q) {
    const int64_t N = p->n_vertices;
    r.N = N;
    r.P = p->n_paths;
    r.K = (int)(N < q->k ? N : q->k);
    r.D = q->D;
    r.schedule = resolve_schedule(q);
    // single-scene propagation defaults to workgroups of 512 rows: the
    // compact-id aggregation ran 2.5-3.9% faster than with 256 (the shift is
    // indifferent); batches keep 256, which their persistent schedule needs
    r.tile = q->tile ? q->tile : 512;
    r.tile_group = q->tile_group;
    r.tape = (q->flags & PG_FLAG_TAPE) != 0;
    r.clusters = (q->flags & PG_FLAG_CLUSTERS) != 0;
    if (r.clusters) {   // no stored edges: the weights are recomputed from the cluster order
        carve_grid(cv, r.g, N, shift_of(q, N));
        r.rec = cv.take<VRec>(N);
        r.b = cv.take<float>(3 * N);
        r.dpt = cv.take<float>(3 * N);
        r.r = cv.take<float>(N);
        r.alpha = cv.take<float>(N);
        r.succ = cv.take<int32_t>(N);
        r.x = cv.take<float>(3 * N);
        r.y = cv.take<float>(3 * N);
        carve_clusters(cv, r.cl, N, q->k);
        carve_cluster_render(cv, r.cr, N);
        if (r.tape) {   // x_0 and y_1..y_D, and the predecessors
            r.pred = cv.take<int32_t>(N);
            r.traj = cv.take<float>((int64_t)(r.D + 1) * 3 * N);
        }
        return;
    }
    const int64_t E = ell_size(N, r.K);   // sliced-ELL storage, padded to whole slices
    carve_grid(cv, r.g, N, shift_of(q, N));
    r.rec = cv.take<VRec>(N);
    r.recp = cv.take<VRec>(N);
    r.col = cv.take<int32_t>(E);
    r.w = cv.take<float>(E);
    r.gw = r.tape ? cv.take<float>(E) : nullptr;
    r.b = cv.take<float>(3 * N);
    r.dpt = cv.take<float>(3 * N);
    r.r = cv.take<float>(N);
    r.alpha = cv.take<float>(N);
    r.succ = cv.take<int32_t>(N);
    r.pred = (r.tape || r.schedule == PG_SCHED_SCATTER) ? cv.take<int32_t>(N) : nullptr;
    r.x = cv.take<float>(3 * N);
    r.y = cv.take<float>(3 * N);
    // decided from the sizes alone: a sizing pass carves from a null base, so
    // no buffer's pointer may decide what is carved
    const bool compact = r.schedule == PG_SCHED_TWO_PASS && ell_k4(r.K) <= 32 && E < ((int64_t)1 << 32);
    if (compact) {
        const int64_t nsl = div_up(N, kSlice);
        r.c16 = cv.take<int16_t>(c16_size(N, r.K));
        r.c16_base = cv.take<uint32_t>(nsl + 1);
        r.c16_cnt = cv.take<uint32_t>(nsl);
        r.c16_part = cv.take<uint32_t>((int64_t)(scan_partials_bytes(nsl) / sizeof(uint32_t)));
        r.c16_ovf = cv.take<int32_t>(E);
    }
    if (r.schedule == PG_SCHED_SHIFTED) {
        r.mcol = cv.take<int32_t>(E);
        r.mw = cv.take<float>(E);
        r.c = cv.take<float>(3 * N);
    }
    r.traj = r.tape ? cv.take<float>((int64_t)(r.D + 1) * 3 * N) : nullptr;
    const int k4 = ell_k4(r.K);
    if (r.tape && (q->flags & PG_FLAG_STORE_Z) && compact && (k4 == 8 || k4 == 12 || k4 == 16))
        r.zt = cv.take<float>((int64_t)r.D * 6 * N);
}

#define PG_TRY(x)                              \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

hipError_t render_setup(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                        hipStream_t s, float** x0_out) {
    const int64_t N = r.N;
    const int K = r.K;
    GridBufs& g = r.g;
    {
        ProfScope ps(s, "grid");
        PG_TRY(run_grid(p, g, r.rec, s, r.recp));
    }
    if (N == 0) {
        if (out && out->row_ptr) PG_TRY(launch_fill(out->row_ptr, sizeof(int64_t), s));
    } else {
        ProfScope ps(s, "knn");
        PG_TRY(launch_knn(N, K, g.shift, g.qs, g.perm, g.inv, g.range, r.col, out ? out->col : nullptr,
                          out ? out->row_ptr : nullptr, g.redo, g.nredo, (q->flags & PG_FLAG_EXACT_KNN) != 0, s));
    }
    const Consts c = make_consts(q, K);
    EdgeOut o{};
    o.ell = 1;
    o.w = r.w;
    o.gw = r.gw;
    o.b = r.b;
    o.dpt = r.dpt;
    o.r = r.r;
    o.alpha = r.alpha;
    o.canon_row = g.perm;
    o.emit = p->l_emit;
    o.dir_pl = p->dir_pl;
    o.l_pl = p->l_pl;
    if (out) {
        o.w_ind = out->w_ind;
        o.w_ph = out->w_ph;
        o.w_env = out->w_env;
        o.b_canon = out->b;
        o.dpt_canon = out->d_pt;
    }
    {
        ProfScope ps(s, "edges");
        PG_TRY(launch_edges(N, c, r.col, r.rec, o, g.flag, s));
    }
    if (r.c16) {
        ProfScope ps(s, "compact_ids");
        PG_TRY(launch_c16_build(N, K, r.col, r.c16, r.c16_cnt, r.c16_base, r.c16_part, r.c16_ovf, s));
    }
    float* x0 = r.tape ? r.traj : r.x;
    PG_TRY(launch_fill_value(r.succ, (size_t)N * 4, 0xffffffffu, s));
    if (r.pred) PG_TRY(launch_fill_value(r.pred, (size_t)N * 4, 0xffffffffu, s));
    PG_TRY(launch_fill(x0, (size_t)N * 12, s));
    {
        ProfScope ps(s, "paths");
        PG_TRY(launch_paths(r.P, N, p->path_offsets, g.inv, r.alpha, r.dpt, r.r, p->l_emit, q->init, r.succ, r.pred, x0,
                            g.flag, s));
    }
    if (r.schedule == PG_SCHED_SCATTER) {
        // path ends are never written by the scatter: they stay 0 in every buffer
        if (r.tape) PG_TRY(launch_fill(r.traj + (size_t)N * 3, (size_t)r.D * N * 12, s));
        else PG_TRY(launch_fill(r.y, (size_t)N * 12, s));
    }
    if (r.schedule == PG_SCHED_SHIFTED) {
        ProfScope ps(s, "shifted_build");
        PG_TRY(launch_shifted_build(N, K, r.succ, r.col, r.w, r.b, r.alpha, r.mcol, r.mw, r.c, s));
    }
    *x0_out = x0;
    return hipSuccess;
}

hipError_t render_iterate(RenderBufs& r, float* x0, hipStream_t s, float** final_x) {
    const int64_t N = r.N;
    const int K = r.K;
    float* cur = x0;
    for (int t = 1; t <= r.D; ++t) {
        float* nxt;
        if (r.tape) nxt = r.traj + (size_t)t * N * 3;
        else if (r.schedule != PG_SCHED_TWO_PASS) nxt = (cur == r.x) ? r.y : r.x;
        else nxt = r.x;
        if (r.schedule == PG_SCHED_SHIFTED) {
            ProfScope ps(s, "spmv_shifted");
            PG_TRY(launch_spmv_shifted(N, K, r.succ, r.mcol, r.mw, r.c, cur, nxt, s));
        } else if (r.schedule == PG_SCHED_SCATTER) {
            ProfScope ps(s, "spmv_scatter");
            PG_TRY(launch_spmv_scatter(N, K, r.col, r.w, cur, r.b, r.alpha, r.pred, nxt, s));
        } else {
            {
                ProfScope ps(s, "spmv");
                if (r.zt)
                    PG_TRY(launch_spmv_c16_tape(N, K, r.c16, r.c16_base, r.c16_ovf, r.w, r.gw, cur, r.b, r.alpha, r.y,
                                                r.zt + (size_t)(t - 1) * N * 6, s, r.tile, r.tile_group));
                else if (r.c16)
                    PG_TRY(launch_spmv_c16(N, K, r.c16, r.c16_base, r.c16_ovf, r.col, r.w, cur, r.b, r.alpha, r.y, s,
                                           r.tile, r.tile_group));
                else
                    PG_TRY(launch_spmv_ell(N, K, r.col, r.w, cur, r.b, r.alpha, nullptr, r.y, s, r.tile,
                                           r.tile_group));
            }
            ProfScope ps(s, "shift");
            PG_TRY(launch_shift(N, r.succ, r.y, nxt, s, r.tile));
        }
        cur = nxt;
    }
    *final_x = cur;
    return hipSuccess;
}

hipError_t render_output(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out,
                         float* image, const float* cur, hipStream_t s) {
    const Consts c = make_consts(q, r.K);
    {
        ProfScope ps(s, "pixels");
        PG_TRY(launch_pixels(*p, c, r.g.inv, r.col, r.w, cur, r.dpt, r.r, r.alpha, image, r.g.flag, s));
    }
    if (out && out->lplus) PG_TRY(launch_permute3(r.N, r.g.perm, cur, out->lplus, 0, s));
    if (out && out->n_far) {   // the escape list's length, widened to int64
        PG_TRY(launch_fill(out->n_far, sizeof(int64_t), s));
        if (r.c16)
            PG_TRY(hipMemcpyAsync(out->n_far, r.c16_base + div_up(r.N, kSlice), sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, s));
    }
    return hipSuccess;
}

hipError_t run_render(const pg_paths* p, const pg_params* q, RenderBufs& r, const pg_graph_out* out, float* image,
                      hipStream_t s, float** final_x) {
    float* x0 = nullptr;
    float* cur = nullptr;
    if (r.clusters) {
        PG_TRY(cluster_setup(p, q, r, out, s, &x0));
        PG_TRY(cluster_iterate(r, q, x0, s, &cur));
        PG_TRY(cluster_output(p, q, r, out, image, cur, s));
        if (final_x) *final_x = cur;
        return hipSuccess;
    }
    PG_TRY(render_setup(p, q, r, out, s, &x0));
    PG_TRY(render_iterate(r, x0, s, &cur));
    PG_TRY(render_output(p, q, r, out, image, cur, s));
    if (final_x) *final_x = cur;
    return hipSuccess;
}

}  // namespace pg
