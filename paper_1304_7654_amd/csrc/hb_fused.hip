// Host side of the fused, batched stage kernel (hb_fused_kernel.hpp): kernel
// arguments, the Runge-Kutta stage sequence, graph capture of whole
// iterations, and the tile lists with their halo tables.
#include "hb_fused_kernel.hpp"

#include <algorithm>
#include <type_traits>

namespace hb {
namespace {

using namespace fk;

}  // namespace

// the variants are instantiated in hb_fused_k*.hip
namespace fk {
#define HB_FUSED_VARIANT(T, MV, BIG) \
    extern template int launch_stage<T, MV, BIG>(hb_grid *, const FusedArgs<T> &, bool, int, hipStream_t);
HB_FUSED_VARIANT(float, false, false)
HB_FUSED_VARIANT(double, false, false)
HB_FUSED_VARIANT(float, true, false)
HB_FUSED_VARIANT(double, true, false)
HB_FUSED_VARIANT(float, false, true)
HB_FUSED_VARIANT(double, false, true)
HB_FUSED_VARIANT(float, true, true)
HB_FUSED_VARIANT(double, true, true)
#undef HB_FUSED_VARIANT
}  // namespace fk

namespace {

template <class T>
FusedArgs<T> make_args(hb_grid *g);

template <>
FusedArgs<float> make_args<float>(hb_grid *g) {
    FusedArgs<float> a{};
    const Consts &c = g->consts;
    a.blks = g->blk_d; a.tiles = g->tiles_d; a.gtab = g->gtab_d; a.n_tiles = g->n_tiles;
    a.SI = g->SI_f; a.dI = g->dI_f; a.SJ = g->SJ_f; a.dJ = g->dJ_f; a.V = g->V_f;
    a.D = g->D_f; a.ffw = g->ffw_f; a.dqinf = g->dqinf_f; a.ffq = g->ffq_d;
    a.partials = g->partials_d; a.status = g->status_d; a.dtau = g->dtau_f;
    a.gamma = (float)c.gamma; a.mu = (float)c.mu; a.kappa = (float)c.kappa;
    a.mu_pr = (float)(c.mu / c.prandtl); a.cfl = (float)c.cfl; a.delta = (float)c.delta_frac;
    a.eps = (float)c.eps;
    a.h2d = c.delta_frac > 0.0 ? (float)(0.5 / c.delta_frac) : 0.0f;
    a.mot = g->motion.tab; a.xp = g->motion.xp; a.yp = g->motion.yp;
    a.xy = g->xy_d; a.C = g->C_d; a.wtab = g->wtab_d; a.gtab64 = g->gtab64_d;
    return a;
}

template <>
FusedArgs<double> make_args<double>(hb_grid *g) {
    FusedArgs<double> a{};
    const Consts &c = g->consts;
    a.blks = g->blk_d; a.tiles = g->tiles_d; a.gtab = g->gtab_d; a.n_tiles = g->n_tiles;
    a.SI = g->SI_d; a.dI = g->dI_d; a.SJ = g->SJ_d; a.dJ = g->dJ_d; a.V = g->V_d;
    a.D = g->D_d; a.ffw = g->ffw_d; a.dqinf = g->dqinf_d; a.ffq = g->ffq_d;
    a.partials = g->partials_d; a.status = g->status_d; a.dtau = g->dtau_d;
    a.gamma = c.gamma; a.mu = c.mu; a.kappa = c.kappa; a.mu_pr = c.mu / c.prandtl; a.cfl = c.cfl;
    a.delta = c.delta_frac; a.eps = c.eps;
    a.h2d = c.delta_frac > 0.0 ? 0.5 / c.delta_frac : 0.0;
    a.mot = g->motion.tab; a.xp = g->motion.xp; a.yp = g->motion.yp;
    a.xy = g->xy_d; a.C = g->C_d; a.wtab = g->wtab_d; a.gtab64 = g->gtab64_d;
    return a;
}

// one stage: k = stage index, input/output buffers chosen by the caller
template <class T>
int stage(hb_grid *g, bool first, int mode, const double *q0, const T *sin, T *sout, double *qout,
          double alpha, int norm, hipStream_t s) {
    FusedArgs<T> a = make_args<T>(g);
    a.q0 = q0; a.sin = sin; a.sout = sout; a.qout = qout; a.alpha = alpha; a.norm = norm;
    if (a.mot) {
        if (g->big) return launch_stage<T, true, true>(g, a, first, mode, s);
        return launch_stage<T, true, false>(g, a, first, mode, s);
    }
    if (g->big) return launch_stage<T, false, true>(g, a, first, mode, s);
    return launch_stage<T, false, false>(g, a, first, mode, s);
}

template <class T>
int one_iteration(hb_grid *g, double *q, T *sa, T *sb, double *resnorm, hipStream_t s) {
    const int ns = g->solver.n_stages;
    const T *in = nullptr;
    for (int k = 0; k < ns; ++k) {
        const bool last = k == ns - 1;
        T *out = (k % 2 == 0) ? sa : sb;
        hipEvent_t end;
        int rc = prof_begin(g, s, &end);
        if (rc) return rc;
        rc = stage<T>(g, k == 0, last ? 2 : 1, q, in, last ? nullptr : out, last ? q : nullptr,
                      g->solver.rk_alpha[k], k == 0, s);
        if (rc) return rc;
        rc = prof_end(end, s);
        if (rc) return rc;
        in = out;
    }
    return launch_norm_finalize(g, g->partials_d, g->n_tiles, resnorm, g->ctr_d, s);
}

template <class T>
int rk_graph(hb_grid *g, double *q, int n_iter, double *resnorm, T *sa, T *sb, hipStream_t s) {
    int rc = launch_reset_ctr(g->ctr_d, s);
    if (rc) return rc;
    if (g->prof) {            // instrumented: stage by stage, no graph
        for (int it = 0; it < n_iter && !rc; ++it) rc = one_iteration<T>(g, q, sa, sb, resnorm, s);
        return rc;
    }
    const int per = std::max(1, g->solver.graph_iters);
    if (!g->graph_exec || g->graph_q != q || g->graph_norm != resnorm || g->graph_iters != per) {
        if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
        g->graph_exec = nullptr;
        if (!g->cap_stream) {
            rc = check_hip(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking), "stream");
            if (rc) return rc;
        }
        rc = check_hip(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal), "capture");
        if (rc) return rc;
        for (int k = 0; k < per && !rc; ++k) rc = one_iteration<T>(g, q, sa, sb, resnorm, g->cap_stream);
        hipGraph_t graph = nullptr;
        const int rc2 = check_hip(hipStreamEndCapture(g->cap_stream, &graph), "end capture");
        if (rc || rc2) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc ? rc : rc2;
        }
        rc = check_hip(hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0), "instantiate");
        (void)hipGraphDestroy(graph);
        if (rc) return rc;
        g->graph_q = q;
        g->graph_norm = resnorm;
        g->graph_iters = per;
    }
    int done = 0;
    for (; done + per <= n_iter; done += per) {
        rc = check_hip(hipGraphLaunch(g->graph_exec, s), "graph launch");
        if (rc) return rc;
    }
    for (; done < n_iter; ++done) {
        rc = one_iteration<T>(g, q, sa, sb, resnorm, s);
        if (rc) return rc;
    }
    return HB_OK;
}

}  // namespace

namespace {
std::vector<Tile> make_tiles(const hb_grid *g, int ti, int order) {
    const int tj = kThreads / ti - 1;        // output rows per tile
    std::vector<Tile> tiles;
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        if (order == 0) {
            for (int j0 = 0; j0 < B.nj; j0 += tj)
                for (int i0 = 0; i0 < B.ni; i0 += ti) tiles.push_back(Tile{b, i0, j0, B.ns, -1});
        } else {
            for (int i0 = 0; i0 < B.ni; i0 += ti)
                for (int j0 = 0; j0 < B.nj; j0 += tj) tiles.push_back(Tile{b, i0, j0, B.ns, -1});
        }
    }
    // heavier tiles first: the static stride then hands every workgroup a
    // similar mix of snapshot counts
    std::stable_sort(tiles.begin(), tiles.end(), [](const Tile &x, const Tile &y) { return x.ns > y.ns; });
    return tiles;
}
}  // namespace

// Largest tile list over the supported shapes (sizes the per-tile partials).
int64_t fused_max_tiles(const hb_grid *g) {
    return (int64_t)std::max(make_tiles(g, 16, 0).size(), make_tiles(g, 32, 0).size());
}

void fused_drop_graph(hb_grid *g) {
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
    g->graph_q = g->graph_norm = nullptr;
}

// Tile list of the given shape (tile_i threads along i: 16 or 32) and order;
// synchronous upload.  Drops a captured graph (it holds the old list).
int fused_build_tiles(hb_grid *g, int tile_i, int order) {
    if (g->solver.n_stages < 2)
        return fail(HB_ERR_UNSUPPORTED, "the fused path needs at least two Runge-Kutta stages");
    if ((tile_i != 16 && tile_i != 32) || (order != 0 && order != 1))
        return fail(HB_ERR_ARG, "tile_i must be 16 or 32 and tile_order 0 or 1");
    std::vector<Tile> tiles = make_tiles(g, tile_i, order);
    // halo source tables of the tiles whose ghost-extended region leaves the
    // block: entry e of a tile describes ext cell e (row-major over the
    // (TI + 4) x (OJ + 4) region, two entries per thread); cells beyond the
    // second ghost layer of a partial tile, and the entries past the region,
    // are far field
    const int ti = tile_i, oj = kThreads / tile_i - 1;
    const int we = ti + 4, ext = (ti + 4) * (oj + 4);
    std::vector<uint32_t> tab, wtab;
    std::vector<uint64_t> tab64;
    for (Tile &t : tiles) {
        const BlockDesc &K = g->blk[t.blk];
        if (t.i0 >= 2 && t.i0 + ti + 2 <= K.ni && t.j0 >= 2 && t.j0 + oj + 2 <= K.nj) continue;
        t.gtab = (int)(tab.size() / 2);
        for (int e = 0; e < 2 * kThreads; ++e) {
            uint32_t x = 0, y = 0;
            uint64_t o64 = 0;
            const int gi = t.i0 + e % we - 2, gj = t.j0 + e / we - 2;
            if (e < ext && gi < K.ni + 2 && gj < K.nj + 2) {
                const GSrc src = ghost_src(g->blk, g->segs, t.blk, gi, gj);
                if (src.cell) {
                    const BlockDesc &S = g->blk[src.b];
                    const int64_t el = S.q_off + (int64_t)src.j * S.ni + src.i;
                    // 64-bit addressing takes the offset from tab64
                    x = g->big ? 0u : (uint32_t)el;
                    y = (uint32_t)(S.ni * S.nj);
                    if (g->big) o64 = (uint64_t)el;
                }
                x |= (uint32_t)src.mir << 31;
            }
            tab.push_back(x);
            tab.push_back(y);
            if (g->big) tab64.push_back(o64);
            // moving no-slip wall image: its wall face (moving grids)
            uint32_t wx = 0, wy = 0;
            if (e < ext && gi < K.ni + 2 && gj < K.nj + 2) {
                const WallFace wf = wall_face(g->blk, g->segs, t.blk, gi, gj);
                if (wf.node >= 0) {
                    const BlockDesc &S = g->blk[wf.blk];
                    wx = (uint32_t)(2 * S.node_off + wf.node);
                    wy = (uint32_t)((S.ni + 1) * (S.nj + 1));
                }
            }
            wtab.push_back(wx);
            wtab.push_back(wy);
        }
    }
    if (2 * g->n_nodes >= ((int64_t)1 << 32))
        return fail(HB_ERR_UNSUPPORTED, "node arrays too large for the batched halo tables");
    hipDeviceProp_t prop;
    int rc = check_hip(hipGetDeviceProperties(&prop, g->device), "device properties");
    if (rc) return rc;
    g->n_cu = prop.multiProcessorCount;
    rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc) return rc;
    fused_drop_graph(g);
    if (g->tiles_d) (void)hipFree(g->tiles_d);
    g->tiles_d = nullptr;
    rc = check_hip(hipMalloc((void **)&g->tiles_d, sizeof(Tile) * tiles.size()), "tiles alloc");
    if (rc) return rc;
    rc = check_hip(hipMemcpy(g->tiles_d, tiles.data(), sizeof(Tile) * tiles.size(),
                             hipMemcpyHostToDevice), "tiles upload");
    if (rc) return rc;
    if (g->gtab_d) (void)hipFree(g->gtab_d);
    g->gtab_d = nullptr;
    rc = check_hip(hipMalloc((void **)&g->gtab_d, sizeof(uint32_t) * std::max<size_t>(2, tab.size())),
                   "halo table alloc");
    if (rc) return rc;
    if (!tab.empty())
        rc = check_hip(hipMemcpy(g->gtab_d, tab.data(), sizeof(uint32_t) * tab.size(),
                                 hipMemcpyHostToDevice), "halo table upload");
    if (rc) return rc;
    if (g->wtab_d) (void)hipFree(g->wtab_d);
    g->wtab_d = nullptr;
    rc = check_hip(hipMalloc((void **)&g->wtab_d, sizeof(uint32_t) * std::max<size_t>(2, wtab.size())),
                   "wall table alloc");
    if (rc) return rc;
    if (!wtab.empty())
        rc = check_hip(hipMemcpy(g->wtab_d, wtab.data(), sizeof(uint32_t) * wtab.size(),
                                 hipMemcpyHostToDevice), "wall table upload");
    if (rc) return rc;
    if (g->gtab64_d) (void)hipFree(g->gtab64_d);
    g->gtab64_d = nullptr;
    if (g->big) {
        rc = check_hip(hipMalloc((void **)&g->gtab64_d, sizeof(uint64_t) * std::max<size_t>(1, tab64.size())),
                       "halo table alloc");
        if (rc) return rc;
        if (!tab64.empty())
            rc = check_hip(hipMemcpy(g->gtab64_d, tab64.data(), sizeof(uint64_t) * tab64.size(),
                                     hipMemcpyHostToDevice), "halo table upload");
        if (rc) return rc;
    }
    g->tile_ti = tile_i;
    g->tile_tj = kThreads / tile_i - 1;
    g->tune_order = order;
    g->n_tiles = (int)tiles.size();
    return HB_OK;
}

// n_iter eager iterations (no graph, no norm output) on q; the mean time of
// one stage launch in milliseconds, from HIP events around the whole run.
int fused_time_iterations(hb_grid *g, double *q, int n_iter, double *ms_per_stage, hipStream_t s) {
    hipEvent_t e0, e1;
    int rc = check_hip(hipEventCreate(&e0), "event");
    if (rc) return rc;
    rc = check_hip(hipEventCreate(&e1), "event");
    if (rc) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    const int prof = g->prof;
    g->prof = 0;
    rc = launch_reset_ctr(g->ctr_d, s);
    rc = rc ? rc : check_hip(hipEventRecord(e0, s), "event record");
    for (int it = 0; it < n_iter && !rc; ++it) {
        if (g->solver.precision == HB_FP32_BULK) rc = one_iteration<float>(g, q, g->sa_f, g->sb_f, nullptr, s);
        else rc = one_iteration<double>(g, q, g->qa_d, g->qb_d, nullptr, s);
    }
    rc = rc ? rc : check_hip(hipEventRecord(e1, s), "event record");
    rc = rc ? rc : check_hip(hipEventSynchronize(e1), "event sync");
    float ms = 0.0f;
    rc = rc ? rc : check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    g->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) *ms_per_stage = (double)ms / std::max(1, n_iter * g->solver.n_stages);
    return rc;
}

int fused_residual(hb_grid *g, const double *q, double *r, hipStream_t s) {
    if (g->solver.precision == HB_FP32_BULK)
        return stage<float>(g, true, 0, q, nullptr, nullptr, r, 0.0, 0, s);
    return stage<double>(g, true, 0, q, nullptr, nullptr, r, 0.0, 0, s);
}

int fused_rk_iterate(hb_grid *g, double *q, int n_iter, double *resnorm, hipStream_t s) {
    if (g->solver.precision == HB_FP32_BULK)
        return rk_graph<float>(g, q, n_iter, resnorm, g->sa_f, g->sb_f, s);
    return rk_graph<double>(g, q, n_iter, resnorm, g->qa_d, g->qb_d, s);
}

}  // namespace hb
