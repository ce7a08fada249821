// C ABI of libhb: argument validation, grid construction (device memory,
// block table, per-snapshot tables, HB matrices, metrics) and dispatch of
// each entry point to the plain or the fused kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hb_internal.hpp"

namespace {
thread_local std::string g_err;
}

namespace hb {

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return HB_OK;
    return fail(e == hipErrorOutOfMemory ? HB_ERR_OOM : HB_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

template <class T>
int dalloc(T **p, int64_t n) {
    *p = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(HB_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return HB_OK;
}

template <class T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_all(hb_grid *g) {
    for (hipEvent_t e : g->prof_ev) (void)hipEventDestroy(e);
    g->prof_ev.clear();
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
    for (int k = 0; k < hb_grid::kSide; ++k) {
        if (g->side[k]) (void)hipStreamDestroy(g->side[k]);
        if (g->join_ev[k]) (void)hipEventDestroy(g->join_ev[k]);
        g->side[k] = nullptr;
        g->join_ev[k] = nullptr;
    }
    if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
    g->fork_ev = nullptr;
    dfree(g->blk_d);
    dfree(g->xy_d);
    dfree(g->SI_d); dfree(g->dI_d); dfree(g->SJ_d); dfree(g->dJ_d);
    dfree(g->V_d); dfree(g->C_d);
    dfree(g->SI_f); dfree(g->dI_f); dfree(g->SJ_f); dfree(g->dJ_f); dfree(g->V_f);
    dfree(g->D_d); dfree(g->D_f);
    dfree(g->ffw_d); dfree(g->ffq_d); dfree(g->dqinf_d);
    dfree(g->ffw_f); dfree(g->ffq_f); dfree(g->dqinf_f);
    dfree(g->ext_d); dfree(g->FI_d); dfree(g->FJ_d); dfree(g->mot_d);
    dfree(g->q0_d); dfree(g->qa_d); dfree(g->qb_d);
    dfree(g->sa_f); dfree(g->sb_f);
    dfree(g->dtau_f); dfree(g->dtau_d);
    dfree(g->partials_d); dfree(g->fpart_d); dfree(g->norm_tmp_d);
    dfree(g->status_d); dfree(g->ctr_d);
    dfree(g->body_off_d); dfree(g->body_ns_d);
    dfree(g->body_ptr_d); dfree(g->body_blk_d);
    dfree(g->tiles_d);
    dfree(g->gtab_d);
    dfree(g->segs_d);
    dfree(g->wtab_d);
    dfree(g->gtab64_d);
    dfree(g->ffc_d);
    dfree(g->cpart_d);
    dfree(g->geo_d);
    dfree(g->vb_d);
    dfree(g->mb_d);
    dfree(g->adj_d);
    dfree(g->AFI_d); dfree(g->AFJ_d); dfree(g->NB_d); dfree(g->WBext_d); dfree(g->adj_part_d);
    dfree(g->fold_ptr_d); dfree(g->fold_b_d); dfree(g->fold_p_d); dfree(g->fold_m_d);
    dfree(g->ff_ptr_d); dfree(g->ff_p_d); dfree(g->ff_m_d);
    dfree(g->ext_adj_d);
    dfree(g->cf_adj_d);
    dfree(g->it_lam0_d); dfree(g->it_qbar_d); dfree(g->it_dtv_d); dfree(g->it_part_d);
    dfree(g->td_r_d); dfree(g->td_acc_d); dfree(g->td_qs_d);
}

bool known_bc(int k) { return k >= HB_BC_WALL && k <= HB_BC_CUT_FARFIELD; }

// sides glued by cut segments: wholly (HB_BC_CUT) or partly
bool glued_kind(int k) { return k == HB_BC_CUT || k == HB_BC_CUT_WALL || k == HB_BC_CUT_FARFIELD; }

// kind of the cells of a glued side that no segment covers (0: none may be)
int rest_kind(int k) {
    return k == HB_BC_CUT_WALL ? HB_BC_WALL : k == HB_BC_CUT_FARFIELD ? HB_BC_FARFIELD : 0;
}

// HB time-derivative matrix, closed form of the odd-N spectral
// differentiation matrix: D[n][m] = (omega/2) (-1)^(n-m) / sin(pi (n-m) / N).
void hb_matrix(int nh, double omega, double *D /* kNsPad x kNsPad */) {
    const int ns = 2 * nh + 1;
    for (int k = 0; k < kNsPad * kNsPad; ++k) D[k] = 0.0;
    for (int n = 0; n < ns; ++n)
        for (int m = 0; m < ns; ++m) {
            if (n == m) continue;
            const int d = n - m;
            const double sgn = (d % 2 == 0) ? 1.0 : -1.0;
            D[n * kNsPad + m] = 0.5 * omega * sgn / std::sin(M_PI * d / ns);
        }
}

}  // namespace

// Per-snapshot tables: free stream at alpha(t_n) and sum_m D[n][m] Q_inf(m).
int upload_snapshot_tables(hb_grid *g) {
    const hb_flow &f = g->flow;
    const double omega = 2.0 * f.k_red * f.mach / f.l_ref;
    std::vector<double> ffw(4 * g->n_snap), ffq(4 * g->n_snap), dq(4 * g->n_snap);
    std::vector<double> D(kNsPad * kNsPad);
    for (const BlockDesc &B : g->blk) {
        hb_matrix(B.nh, omega, D.data());
        for (int n = 0; n < B.ns; ++n) {
            const double a = f.alpha0 + f.alpha_amp * std::sin(2.0 * M_PI * n / B.ns);
            const double u = f.mach * std::cos(a), v = f.mach * std::sin(a), p = 1.0 / f.gamma;
            double *w = &ffw[4 * (B.snap_off + n)];
            double *q = &ffq[4 * (B.snap_off + n)];
            w[0] = 1.0; w[1] = u; w[2] = v; w[3] = p;
            q[0] = 1.0; q[1] = u; q[2] = v; q[3] = p / (f.gamma - 1.0) + 0.5 * (u * u + v * v);
        }
        for (int n = 0; n < B.ns; ++n)
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int m = 0; m < B.ns; ++m) s += D[n * kNsPad + m] * ffq[4 * (B.snap_off + m) + c];
                dq[4 * (B.snap_off + n) + c] = s;
            }
    }
    std::vector<float> tmp(4 * g->n_snap);
    int rc = check_hip(hipMemcpy(g->ffw_d, ffw.data(), sizeof(double) * ffw.size(), hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->ffq_d, ffq.data(), sizeof(double) * ffq.size(), hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->dqinf_d, dq.data(), sizeof(double) * dq.size(), hipMemcpyHostToDevice), "upload");
    for (size_t k = 0; k < tmp.size() && !rc; ++k) tmp[k] = (float)ffw[k];
    rc = rc ? rc : check_hip(hipMemcpy(g->ffw_f, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice), "upload");
    for (size_t k = 0; k < tmp.size() && !rc; ++k) tmp[k] = (float)ffq[k];
    rc = rc ? rc : check_hip(hipMemcpy(g->ffq_f, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice), "upload");
    for (size_t k = 0; k < tmp.size() && !rc; ++k) tmp[k] = (float)dq[k];
    rc = rc ? rc : check_hip(hipMemcpy(g->dqinf_f, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice), "upload");
    return rc;
}

int prof_begin(hb_grid *g, hipStream_t s, hipEvent_t *end) {
    *end = nullptr;
    if (!g->prof) return HB_OK;
    while (g->prof_ev.size() < g->prof_used + 2) {
        hipEvent_t e;
        int rc = check_hip(hipEventCreate(&e), "event create");
        if (rc) return rc;
        g->prof_ev.push_back(e);
    }
    hipEvent_t b = g->prof_ev[g->prof_used];
    *end = g->prof_ev[g->prof_used + 1];
    g->prof_used += 2;
    return check_hip(hipEventRecord(b, s), "event record");
}

int prof_end(hipEvent_t end, hipStream_t s) {
    if (!end) return HB_OK;
    return check_hip(hipEventRecord(end, s), "event record");
}

}  // namespace hb

using namespace hb;

extern "C" {

const char *hb_last_error(void) { return g_err.c_str(); }

int hb_grid_create(const hb_block *blocks, int32_t nblocks, const hb_cut *cuts, int32_t ncuts,
                   const hb_flow *flow, const hb_solver *solver, hb_grid **out) {
    g_err.clear();
    if (!out) return fail(HB_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!blocks || nblocks < 1) return fail(HB_ERR_ARG, "need at least one block");
    if (!flow || !solver) return fail(HB_ERR_ARG, "flow and solver must not be NULL");
    if (ncuts < 0 || (ncuts > 0 && !cuts)) return fail(HB_ERR_ARG, "bad cut list");
    if (!(flow->mach > 0) || !(flow->reynolds > 0) || !(flow->prandtl > 0) ||
        !(flow->gamma > 1) || !(flow->l_ref > 0) || !std::isfinite(flow->alpha0) ||
        !std::isfinite(flow->alpha_amp) || !std::isfinite(flow->k_red) || flow->k_red < 0)
        return fail(HB_ERR_ARG, "invalid flow settings");
    if (solver->n_stages < 1 || solver->n_stages > 8 || !(solver->cfl > 0) ||
        (solver->precision != HB_FP64 && solver->precision != HB_FP32_BULK) ||
        !(solver->entropy_delta >= 0) || !(solver->limiter_eps > 0) || solver->graph_iters < 1 ||
        (solver->batched < 0 || solver->batched > 2))
        return fail(HB_ERR_ARG, "invalid solver settings");
    if (solver->precision == HB_FP32_BULK && !solver->batched)
        return fail(HB_ERR_ARG, "FP32-bulk precision needs the batched (fused) path");
    int nbody = 0;
    for (int b = 0; b < nblocks; ++b) {
        const hb_block &B = blocks[b];
        char msg[160];
        if (B.ni < 4 || B.nj < 4) {
            std::snprintf(msg, sizeof msg, "block %d: ni, nj must be >= 4", b);
            return fail(HB_ERR_ARG, msg);
        }
        if ((int64_t)B.ni * B.nj > (int64_t)1 << 24) {
            std::snprintf(msg, sizeof msg, "block %d: too many cells", b);
            return fail(HB_ERR_ARG, msg);
        }
        if (B.n_harm < 0 || B.n_harm > 4) {
            std::snprintf(msg, sizeof msg, "block %d: n_harm must be in [0, 4]", b);
            return fail(HB_ERR_ARG, msg);
        }
        if (!B.xy) {
            std::snprintf(msg, sizeof msg, "block %d: xy is NULL", b);
            return fail(HB_ERR_ARG, msg);
        }
        for (int s = 0; s < 4; ++s)
            if (!known_bc(B.bc[s]) || (B.bc[s] == HB_BC_WAKECUT && s != 2)) {
                std::snprintf(msg, sizeof msg, "block %d: bad boundary kind on side %d", b, s);
                return fail(HB_ERR_ARG, msg);
            }
        if ((B.bc[0] == HB_BC_PERIODIC) != (B.bc[1] == HB_BC_PERIODIC) ||
            (B.bc[2] == HB_BC_PERIODIC) != (B.bc[3] == HB_BC_PERIODIC)) {
            std::snprintf(msg, sizeof msg, "block %d: periodic sides must come in pairs", b);
            return fail(HB_ERR_ARG, msg);
        }
        if (B.wake_ncells < 0 || B.wake_ncells > B.ni / 2 ||
            (B.wake_ncells > 0 && B.bc[2] != HB_BC_WAKECUT)) {
            std::snprintf(msg, sizeof msg, "block %d: bad wake_ncells", b);
            return fail(HB_ERR_ARG, msg);
        }
        if (B.body_id < 0 || B.body_id >= nblocks) {
            std::snprintf(msg, sizeof msg, "block %d: bad body_id", b);
            return fail(HB_ERR_ARG, msg);
        }
        if (B.body_id + 1 > nbody) nbody = B.body_id + 1;
        // positive areas (FP64, host)
        const int W = B.ni + 1;
        const int64_t nn = (int64_t)W * (B.nj + 1);
        const double *x = B.xy, *y = B.xy + nn;
        for (int j = 0; j < B.nj; ++j)
            for (int i = 0; i < B.ni; ++i) {
                const double x1 = x[j * W + i], y1 = y[j * W + i];
                const double x2 = x[j * W + i + 1], y2 = y[j * W + i + 1];
                const double x3 = x[(j + 1) * W + i + 1], y3 = y[(j + 1) * W + i + 1];
                const double x4 = x[(j + 1) * W + i], y4 = y[(j + 1) * W + i];
                const double v = 0.5 * ((x3 - x1) * (y4 - y2) - (y3 - y1) * (x4 - x2));
                if (!(v > 0.0)) {
                    std::snprintf(msg, sizeof msg, "block %d: cell (%d, %d) has area %g <= 0", b, i,
                                  j, v);
                    return fail(HB_ERR_ARG, msg);
                }
            }
    }
    std::vector<int> body_nh(nbody, -1);
    for (int b = 0; b < nblocks; ++b) {
        int &h = body_nh[blocks[b].body_id];
        if (h >= 0 && h != blocks[b].n_harm) return fail(HB_ERR_ARG, "blocks of one body differ in n_harm");
        h = blocks[b].n_harm;
    }
    for (int k = 0; k < nbody; ++k)
        if (body_nh[k] < 0) return fail(HB_ERR_ARG, "body ids must be numbered without gaps");
    // cuts: segments of block sides (any two sides, possibly reversed); every
    // side of kind HB_BC_CUT covered by its segments exactly once, the partly
    // glued kinds at most once
    std::vector<std::vector<CutSeg>> side_segs(4 * (size_t)nblocks);
    for (int c = 0; c < ncuts; ++c) {
        const hb_cut k = cuts[c];
        if (k.blk_a < 0 || k.blk_a >= nblocks || k.blk_b < 0 || k.blk_b >= nblocks ||
            k.side_a < 0 || k.side_a > 3 || k.side_b < 0 || k.side_b > 3 ||
            (k.reversed != 0 && k.reversed != 1))
            return fail(HB_ERR_ARG, "bad cut");
        const hb_block &A = blocks[k.blk_a], &B = blocks[k.blk_b];
        const int la = k.side_a < 2 ? A.nj : A.ni;
        const int lb = k.side_b < 2 ? B.nj : B.ni;
        if (k.len < 1 || k.start_a < 0 || k.start_b < 0 ||
            (int64_t)k.start_a + k.len > la || (int64_t)k.start_b + k.len > lb)
            return fail(HB_ERR_ARG, "cut segment outside its block sides");
        if (!glued_kind(A.bc[k.side_a]) || !glued_kind(B.bc[k.side_b]))
            return fail(HB_ERR_ARG, "cut sides must have boundary kind HB_BC_CUT, HB_BC_CUT_WALL or "
                                    "HB_BC_CUT_FARFIELD");
        if (A.n_harm != B.n_harm) return fail(HB_ERR_ARG, "glued blocks must have equal n_harm");
        side_segs[4 * k.blk_a + k.side_a].push_back(
            CutSeg{k.start_a, k.len, k.blk_b, k.side_b, k.start_b, k.reversed});
        side_segs[4 * k.blk_b + k.side_b].push_back(
            CutSeg{k.start_b, k.len, k.blk_a, k.side_a, k.start_a, k.reversed});
    }
    for (int b = 0; b < nblocks; ++b)
        for (int s = 0; s < 4; ++s) {
            const int kind = blocks[b].bc[s];
            if (!glued_kind(kind)) continue;
            std::vector<CutSeg> &v = side_segs[4 * b + s];
            std::sort(v.begin(), v.end(), [](const CutSeg &x, const CutSeg &y) { return x.start < y.start; });
            int pos = 0;
            for (const CutSeg &q : v) {
                if (q.start < pos || (kind == HB_BC_CUT && q.start != pos))
                    return fail(HB_ERR_ARG, kind == HB_BC_CUT
                                                ? "the cuts of a HB_BC_CUT side must cover it exactly once"
                                                : "the cuts of a partly glued side overlap");
                pos = q.start + q.len;
            }
            if (kind == HB_BC_CUT && pos != (s < 2 ? blocks[b].nj : blocks[b].ni))
                return fail(HB_ERR_ARG, "the cuts of a HB_BC_CUT side must cover it exactly once");
        }
    std::vector<CutSeg> seg_table;
    std::vector<BlockDesc> cut_desc(nblocks);     // ni, nj, bc, wake and segment ranges
    for (int b = 0; b < nblocks; ++b) {
        BlockDesc &D = cut_desc[b];
        std::memset(&D, 0, sizeof D);
        D.ni = blocks[b].ni;
        D.nj = blocks[b].nj;
        D.wake = blocks[b].wake_ncells;
        for (int s = 0; s < 4; ++s) {
            // glued sides are HB_BC_CUT below, with the kind of their uncovered cells
            D.bc[s] = glued_kind(blocks[b].bc[s]) ? HB_BC_CUT : blocks[b].bc[s];
            D.rest[s] = rest_kind(blocks[b].bc[s]);
            D.seg_off[s] = (int32_t)seg_table.size();
            D.seg_cnt[s] = (int32_t)side_segs[4 * b + s].size();
            seg_table.insert(seg_table.end(), side_segs[4 * b + s].begin(), side_segs[4 * b + s].end());
        }
    }
    if (!ghosts_resolve(cut_desc, seg_table))
        return fail(HB_ERR_ARG, "the cuts leave ghost cells that do not resolve (cuts around a "
                                "singular corner)");

    // ---- device work starts here --------------------------------------
    hb_grid *g = new (std::nothrow) hb_grid();
    if (!g) return fail(HB_ERR_OOM, "host allocation failed");
    int rc = check_hip(hipGetDevice(&g->device), "hipGetDevice");
    if (rc) {
        delete g;
        return rc;
    }
    g->nblocks = nblocks;
    g->nbody = nbody;
    g->flow = *flow;
    g->solver = *solver;
    const double mu = flow->mach * flow->l_ref / flow->reynolds;
    g->consts = Consts{flow->gamma, mu, mu / ((flow->gamma - 1.0) * flow->prandtl), flow->prandtl,
                       solver->cfl, solver->entropy_delta, solver->limiter_eps, 1.0 / flow->gamma};
    const double omega = 2.0 * flow->k_red * flow->mach / flow->l_ref;
    g->blk.resize(nblocks);
    g->segs = seg_table;
    int64_t part = 0;
    for (int b = 0; b < nblocks; ++b) {
        const hb_block &S = blocks[b];
        BlockDesc &B = g->blk[b];
        std::memset(&B, 0, sizeof B);
        B.ni = S.ni; B.nj = S.nj; B.nh = S.n_harm; B.ns = 2 * S.n_harm + 1;
        for (int s = 0; s < 4; ++s) {
            B.bc[s] = cut_desc[b].bc[s];
            B.rest[s] = cut_desc[b].rest[s];
            B.seg_off[s] = cut_desc[b].seg_off[s];
            B.seg_cnt[s] = cut_desc[b].seg_cnt[s];
        }
        B.wake = S.wake_ncells;
        B.body = S.body_id;
        B.snap_off = g->n_snap;
        B.d_off = b * kNsPad * kNsPad;
        B.q_off = g->n_state;
        B.cell_off = g->n_cells;
        B.node_off = g->n_nodes;
        B.fi_off = g->n_fi;
        B.fj_off = g->n_fj;
        B.ext_off = g->n_ext;
        B.fiq_off = g->n_fiq;
        B.fjq_off = g->n_fjq;
        B.part_off = part;
        B.afi_off = g->n_afi;
        B.afj_off = g->n_afj;
        B.nodeq_off = g->n_nodeq;
        B.omega_nh = omega * S.n_harm;
        const int64_t cells = (int64_t)S.ni * S.nj;
        g->n_snap += B.ns;
        g->n_state += (int64_t)B.ns * 4 * cells;
        g->n_cells += cells;
        g->n_nodes += (int64_t)(S.ni + 1) * (S.nj + 1);
        g->n_fi += (int64_t)(S.ni + 1) * S.nj;
        g->n_fj += (int64_t)S.ni * (S.nj + 1);
        g->n_ext += (int64_t)B.ns * 4 * (S.ni + 4) * (S.nj + 4);
        g->n_fiq += (int64_t)B.ns * 4 * (S.ni + 1) * S.nj;
        g->n_fjq += (int64_t)B.ns * 4 * S.ni * (S.nj + 1);
        g->total_cs += (int64_t)B.ns * cells;
        g->n_afi += (int64_t)B.ns * kAF * (S.ni + 1) * S.nj;
        g->n_afj += (int64_t)B.ns * kAF * S.ni * (S.nj + 1);
        g->n_nodeq += (int64_t)B.ns * 3 * (S.ni + 1) * (S.nj + 1);
        part += plain_partials(B);
    }
    g->body_ns.resize(nbody);
    g->body_off.resize(nbody);
    for (int k = 0; k < nbody; ++k) {
        g->body_ns[k] = 2 * body_nh[k] + 1;
        g->body_off[k] = (int)g->n_forces;
        g->n_forces += 3 * g->body_ns[k];
    }
    const bool plain = !solver->batched;
    const bool f32 = solver->precision == HB_FP32_BULK;
    // the batched kernel's halo loads: 32-bit byte offsets while every byte
    // offset into the FP64 state fits, else (or on request) 64-bit
    g->big = !plain && (solver->batched == 2 || g->n_state * (int64_t)sizeof(double) >= ((int64_t)1 << 32));
    rc = dalloc(&g->blk_d, nblocks);
    rc = rc ? rc : dalloc(&g->xy_d, 2 * g->n_nodes);
    rc = rc ? rc : dalloc(&g->SI_d, 2 * g->n_fi);
    rc = rc ? rc : dalloc(&g->dI_d, 2 * g->n_fi);
    rc = rc ? rc : dalloc(&g->SJ_d, 2 * g->n_fj);
    rc = rc ? rc : dalloc(&g->dJ_d, 2 * g->n_fj);
    rc = rc ? rc : dalloc(&g->V_d, g->n_cells);
    rc = rc ? rc : dalloc(&g->C_d, 2 * g->n_cells);
    rc = rc ? rc : dalloc(&g->SI_f, 2 * g->n_fi);
    rc = rc ? rc : dalloc(&g->dI_f, 2 * g->n_fi);
    rc = rc ? rc : dalloc(&g->SJ_f, 2 * g->n_fj);
    rc = rc ? rc : dalloc(&g->dJ_f, 2 * g->n_fj);
    rc = rc ? rc : dalloc(&g->V_f, g->n_cells);
    rc = rc ? rc : dalloc(&g->D_d, (int64_t)nblocks * kNsPad * kNsPad);
    rc = rc ? rc : dalloc(&g->D_f, (int64_t)nblocks * kNsPad * kNsPad);
    rc = rc ? rc : dalloc(&g->ffw_d, 4 * g->n_snap);
    rc = rc ? rc : dalloc(&g->ffq_d, 4 * g->n_snap);
    rc = rc ? rc : dalloc(&g->dqinf_d, 4 * g->n_snap);
    rc = rc ? rc : dalloc(&g->ffw_f, 4 * g->n_snap);
    rc = rc ? rc : dalloc(&g->ffq_f, 4 * g->n_snap);
    rc = rc ? rc : dalloc(&g->dqinf_f, 4 * g->n_snap);
    if (plain) {
        rc = rc ? rc : dalloc(&g->ext_d, g->n_ext);
        rc = rc ? rc : dalloc(&g->FI_d, g->n_fiq);
        rc = rc ? rc : dalloc(&g->FJ_d, g->n_fjq);
    }
    if (!f32) {
        rc = rc ? rc : dalloc(&g->qa_d, g->n_state);
        rc = rc ? rc : dalloc(&g->qb_d, g->n_state);
        if (!plain) rc = rc ? rc : dalloc(&g->dtau_d, g->n_state / 4);
    } else {
        rc = rc ? rc : dalloc(&g->sa_f, g->n_state);
        rc = rc ? rc : dalloc(&g->sb_f, g->n_state);
        if (!plain) rc = rc ? rc : dalloc(&g->dtau_f, g->n_state / 4);
    }
    for (const BlockDesc &B : g->blk) g->fchunks = std::max(g->fchunks, (B.ni + 255) / 256);
    rc = rc ? rc : dalloc(&g->fpart_d, (int64_t)nblocks * kMaxNs * g->fchunks * 3);
    rc = rc ? rc : dalloc(&g->status_d, 1);
    rc = rc ? rc : dalloc(&g->ctr_d, 1);
    rc = rc ? rc : dalloc(&g->body_off_d, nbody);
    rc = rc ? rc : dalloc(&g->body_ns_d, nbody);
    rc = rc ? rc : dalloc(&g->body_ptr_d, nbody + 1);
    rc = rc ? rc : dalloc(&g->body_blk_d, nblocks);
    if (!rc && !plain) rc = fused_build_tiles(g, 16, 0);
    g->n_partials = plain ? part : fused_max_tiles(g);
    rc = rc ? rc : dalloc(&g->partials_d, g->n_partials);
    if (rc) {
        free_all(g);
        delete g;
        return rc;
    }
    // uploads
    std::vector<double> xy(2 * g->n_nodes);
    for (int b = 0; b < nblocks; ++b) {
        const int64_t nn = (int64_t)(blocks[b].ni + 1) * (blocks[b].nj + 1);
        std::memcpy(&xy[2 * g->blk[b].node_off], blocks[b].xy, sizeof(double) * 2 * nn);
    }
    std::vector<double> D((size_t)nblocks * kNsPad * kNsPad);
    std::vector<float> Df(D.size());
    for (int b = 0; b < nblocks; ++b) hb_matrix(g->blk[b].nh, omega, &D[(size_t)b * kNsPad * kNsPad]);
    for (size_t k = 0; k < D.size(); ++k) Df[k] = (float)D[k];
    if (!rc && !g->segs.empty()) {
        rc = dalloc(&g->segs_d, (int64_t)g->segs.size());
        rc = rc ? rc : check_hip(hipMemcpy(g->segs_d, g->segs.data(), sizeof(CutSeg) * g->segs.size(),
                                           hipMemcpyHostToDevice), "upload");
    }
    for (BlockDesc &B : g->blk) B.segs = g->segs_d;
    rc = rc ? rc : check_hip(hipMemcpy(g->blk_d, g->blk.data(), sizeof(BlockDesc) * nblocks, hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->xy_d, xy.data(), sizeof(double) * xy.size(), hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->D_d, D.data(), sizeof(double) * D.size(), hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->D_f, Df.data(), sizeof(float) * Df.size(), hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->body_off_d, g->body_off.data(), sizeof(int) * nbody, hipMemcpyHostToDevice), "upload");
    rc = rc ? rc : check_hip(hipMemcpy(g->body_ns_d, g->body_ns.data(), sizeof(int) * nbody, hipMemcpyHostToDevice), "upload");
    {
        std::vector<int> ptr(nbody + 1, 0), blk;
        for (int k = 0; k < nbody; ++k) {
            for (int b = 0; b < nblocks; ++b)
                if (g->blk[b].body == k) blk.push_back(b);
            ptr[k + 1] = (int)blk.size();
        }
        rc = rc ? rc : check_hip(hipMemcpy(g->body_ptr_d, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice), "upload");
        rc = rc ? rc : check_hip(hipMemcpy(g->body_blk_d, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice), "upload");
    }
    rc = rc ? rc : check_hip(hipMemset(g->status_d, 0, sizeof(int)), "memset");
    rc = rc ? rc : check_hip(hipMemset(g->fpart_d, 0, sizeof(double) * nblocks * kMaxNs * g->fchunks * 3), "memset");
    rc = rc ? rc : upload_snapshot_tables(g);
    rc = rc ? rc : launch_metrics(g, nullptr);
    rc = rc ? rc : check_hip(hipDeviceSynchronize(), "metrics");
    if (rc) {
        free_all(g);
        delete g;
        return rc;
    }
    *out = g;
    return HB_OK;
}

int hb_grid_destroy(hb_grid *g) {
    if (!g) return HB_OK;
    (void)hipDeviceSynchronize();
    free_all(g);
    delete g;
    return HB_OK;
}

int64_t hb_state_size(const hb_grid *g) { return g ? g->n_state : -1; }
int64_t hb_forces_size(const hb_grid *g) { return g ? g->n_forces : -1; }
int64_t hb_xy_size(const hb_grid *g) { return g ? 2 * g->n_nodes : -1; }

int hb_residual(hb_grid *g, const double *q, double *r, void *stream) {
    g_err.clear();
    if (!g || !q || !r) return fail(HB_ERR_ARG, "NULL argument");
    if (q == r) return fail(HB_ERR_ARG, "q and r must not alias");
    hipStream_t s = (hipStream_t)stream;
    if (g->solver.batched) return fused_residual(g, q, r, s);
    return plain_residual(g, q, r, s);
}

int hb_rk_iterate(hb_grid *g, double *q, int32_t n_iter, double *resnorm, double *forces,
                  void *stream) {
    g_err.clear();
    if (!g || !q) return fail(HB_ERR_ARG, "NULL argument");
    if (n_iter < 0) return fail(HB_ERR_ARG, "n_iter must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    int rc = HB_OK;
    if (n_iter > 0)
        rc = g->solver.batched ? fused_rk_iterate(g, q, n_iter, resnorm, s)
                               : plain_rk_iterate(g, q, n_iter, resnorm, s);
    if (!rc && forces) rc = launch_forces(g, q, forces, s);
    return rc;
}

int hb_forces(hb_grid *g, const double *q, double *cf, void *stream) {
    g_err.clear();
    if (!g || !q || !cf) return fail(HB_ERR_ARG, "NULL argument");
    return launch_forces(g, q, cf, (hipStream_t)stream);
}

int hb_residual_adjoint(hb_grid *g, const double *q, const double *rbar, double *qbar,
                        double *xybar, double *flowbar, void *stream) {
    g_err.clear();
    if (!g || !q || !rbar || !qbar) return fail(HB_ERR_ARG, "NULL argument");
    if (qbar == q || qbar == rbar) return fail(HB_ERR_ARG, "qbar must not alias q or rbar");
    if (g->solver.precision != HB_FP64)
        return fail(HB_ERR_UNSUPPORTED, "the adjoint is FP64 only");
    return launch_residual_adjoint(g, q, rbar, qbar, xybar, flowbar, (hipStream_t)stream);
}

int hb_forces_adjoint(hb_grid *g, const double *q, const double *cfbar, double *qbar,
                      double *xybar, double *flowbar, void *stream) {
    g_err.clear();
    if (!g || !q || !cfbar || !qbar) return fail(HB_ERR_ARG, "NULL argument");
    if (qbar == q) return fail(HB_ERR_ARG, "qbar must not alias q");
    return launch_forces_adjoint(g, q, cfbar, qbar, xybar, flowbar, (hipStream_t)stream);
}

int hb_adjoint_iterate(hb_grid *g, const double *q, double *lambda, const double *gq,
                       int32_t n_iter, double *resnorm, void *stream) {
    g_err.clear();
    if (!g || !q || !lambda || !gq) return fail(HB_ERR_ARG, "NULL argument");
    if (n_iter < 0) return fail(HB_ERR_ARG, "n_iter must be >= 0");
    if (lambda == q || lambda == gq) return fail(HB_ERR_ARG, "lambda must not alias q or gq");
    if (g->solver.precision != HB_FP64)
        return fail(HB_ERR_UNSUPPORTED, "the adjoint is FP64 only");
    return launch_adjoint_iterate(g, q, lambda, gq, n_iter, resnorm, (hipStream_t)stream);
}

int hb_prepare(hb_grid *g, int32_t what) {
    g_err.clear();
    if (!g) return fail(HB_ERR_ARG, "NULL grid");
    const int32_t known = HB_PREPARE_ADJOINT | HB_PREPARE_ADJOINT_ITERATE | HB_PREPARE_TD;
    if (what & ~known) return fail(HB_ERR_ARG, "unknown hb_prepare bits");
    if ((what & HB_PREPARE_ADJOINT_ITERATE) && g->solver.precision != HB_FP64)
        return fail(HB_ERR_UNSUPPORTED, "the adjoint iteration is FP64 only");
    int rc = HB_OK;
    if (what & (HB_PREPARE_ADJOINT | HB_PREPARE_ADJOINT_ITERATE))
        rc = adjoint_prepare(g, (what & HB_PREPARE_ADJOINT_ITERATE) != 0);
    if (!rc && (what & HB_PREPARE_TD)) rc = td_prepare(g);
    return rc;
}

int hb_save_state(hb_grid *g, const double *q, int64_t iteration, const char *path, void *stream) {
    g_err.clear();
    if (!g || !q || !path) return fail(HB_ERR_ARG, "NULL argument");
    return io_save(g, q, iteration, path, (hipStream_t)stream);
}

int hb_load_state(hb_grid *g, double *q, int64_t *iteration, const char *path, void *stream) {
    g_err.clear();
    if (!g || !q || !path) return fail(HB_ERR_ARG, "NULL argument");
    return io_load(g, q, iteration, path, (hipStream_t)stream);
}

int hb_save_solution(hb_grid *g, const double *q, const char *prefix, void *stream) {
    g_err.clear();
    if (!g || !q || !prefix || !prefix[0]) return fail(HB_ERR_ARG, "NULL argument");
    return io_save_solution(g, q, prefix, (hipStream_t)stream);
}

int hb_td_march(hb_grid *g, double *q, double t0, double dt, int32_t n_steps, void *stream) {
    g_err.clear();
    if (!g || !q) return fail(HB_ERR_ARG, "NULL argument");
    if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
        return fail(HB_ERR_ARG, "need n_steps >= 0, finite t0 and dt > 0");
    for (const BlockDesc &B : g->blk)
        if (B.nh != 0) return fail(HB_ERR_UNSUPPORTED, "the time-domain march needs n_harm = 0 in every block");
    return launch_td_march(g, q, t0, dt, n_steps, (hipStream_t)stream);
}

int hb_td_march_noalloc(hb_grid *g, double *q, double t0, double dt, int32_t n_steps,
                        void *stream) {
    g_err.clear();
    if (!g || !q) return fail(HB_ERR_ARG, "NULL argument");
    if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
        return fail(HB_ERR_ARG, "need n_steps >= 0, finite t0 and dt > 0");
    for (const BlockDesc &B : g->blk)
        if (B.nh != 0) return fail(HB_ERR_UNSUPPORTED, "the time-domain march needs n_harm = 0 in every block");
    return launch_td_march_noalloc(g, q, t0, dt, n_steps, (hipStream_t)stream);
}

int hb_autotune(hb_grid *g, const double *q, const char *cache_path, int32_t force,
                hb_tuning *out, void *stream) {
    g_err.clear();
    if (!g || !q) return fail(HB_ERR_ARG, "NULL argument");
    if (!g->solver.batched) return fail(HB_ERR_UNSUPPORTED, "tuning applies to batched grids");
    return tune_run(g, q, cache_path, force, out, (hipStream_t)stream);
}

int hb_set_tuning(hb_grid *g, const hb_tuning *t) {
    g_err.clear();
    if (!g || !t) return fail(HB_ERR_ARG, "NULL argument");
    if (!g->solver.batched) return fail(HB_ERR_UNSUPPORTED, "tuning applies to batched grids");
    return tune_set(g, t);
}

int hb_get_tuning(const hb_grid *g, hb_tuning *t) {
    g_err.clear();
    if (!g || !t) return fail(HB_ERR_ARG, "NULL argument");
    if (!g->solver.batched) return fail(HB_ERR_UNSUPPORTED, "tuning applies to batched grids");
    return tune_get(g, t);
}

int hb_set_xy(hb_grid *g, const double *xy, void *stream) {
    g_err.clear();
    if (!g || !xy) return fail(HB_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipMemcpyAsync(g->xy_d, xy, sizeof(double) * 2 * g->n_nodes,
                                      hipMemcpyDeviceToDevice, s), "xy copy");
    return rc ? rc : launch_metrics(g, s);
}

int hb_set_alpha0(hb_grid *g, double alpha0) {
    g_err.clear();
    if (!g || !std::isfinite(alpha0)) return fail(HB_ERR_ARG, "bad argument");
    int rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc) return rc;
    g->flow.alpha0 = alpha0;
    return upload_snapshot_tables(g);
}

int hb_set_motion(hb_grid *g, const hb_motion *m) {
    g_err.clear();
    if (!g) return fail(HB_ERR_ARG, "NULL grid");
    if (m && !(std::isfinite(m->pitch_amp) && std::isfinite(m->pitch_phase) &&
               std::isfinite(m->heave_amp) && std::isfinite(m->x_pivot) && std::isfinite(m->y_pivot)))
        return fail(HB_ERR_ARG, "non-finite motion");
    int rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc) return rc;
    if (!m || (m->pitch_amp == 0.0 && m->heave_amp == 0.0)) {
        fused_drop_graph(g);     // a captured iteration holds the moving-grid kernels
        g->motion = Motion{nullptr, 0.0, 0.0};
        return HB_OK;
    }
    for (const BlockDesc &B : g->blk)
        for (int s = 0; s < 2; ++s)
            if (B.bc[s] == HB_BC_WALL || (B.bc[s] == HB_BC_CUT && B.rest[s] == HB_BC_WALL))
                return fail(HB_ERR_UNSUPPORTED, "moving grids: walls only on j sides");
    if (!g->mot_d) {
        rc = dalloc(&g->mot_d, (int64_t)kMotionW * g->n_snap);
        if (rc) return rc;
    }
    const hb_flow &f = g->flow;
    const double omega = 2.0 * f.k_red * f.mach / f.l_ref;
    std::vector<double> tab((size_t)kMotionW * g->n_snap, 0.0);
    for (const BlockDesc &B : g->blk)
        for (int n = 0; n < B.ns; ++n) {
            const double ph = 2.0 * M_PI * n / B.ns;
            const double th = m->pitch_amp * std::sin(ph + m->pitch_phase);
            double *t = &tab[(size_t)kMotionW * (B.snap_off + n)];
            t[0] = std::cos(th);
            t[1] = std::sin(th);
            t[2] = omega * m->pitch_amp * std::cos(ph + m->pitch_phase);
            t[3] = m->heave_amp * std::sin(ph);
            t[4] = omega * m->heave_amp * std::cos(ph);
        }
    rc = check_hip(hipMemcpy(g->mot_d, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice),
                   "motion upload");
    if (rc) return rc;
    fused_drop_graph(g);         // a captured iteration holds the old kernels and pivot
    g->motion = Motion{g->mot_d, m->x_pivot, m->y_pivot};
    g->motion_par = *m;
    return HB_OK;
}

int hb_profile_stages(hb_grid *g, int32_t enable) {
    g_err.clear();
    if (!g) return fail(HB_ERR_ARG, "NULL grid");
    g->prof = enable ? 1 : 0;
    return HB_OK;
}

int hb_stage_stats(hb_grid *g, double *total_ms, int64_t *stages) {
    g_err.clear();
    if (!g) return fail(HB_ERR_ARG, "NULL grid");
    double ms = 0.0;
    for (size_t k = 0; k + 1 < g->prof_used; k += 2) {
        int rc = check_hip(hipEventSynchronize(g->prof_ev[k + 1]), "event sync");
        if (rc) return rc;
        float t = 0.0f;
        rc = check_hip(hipEventElapsedTime(&t, g->prof_ev[k], g->prof_ev[k + 1]), "elapsed");
        if (rc) return rc;
        ms += t;
    }
    if (total_ms) *total_ms = ms;
    if (stages) *stages = (int64_t)(g->prof_used / 2);
    g->prof_used = 0;
    return HB_OK;
}

int hb_get_status(hb_grid *g) {
    g_err.clear();
    if (!g) return fail(HB_ERR_ARG, "NULL grid");
    int rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc) return rc;
    int st = 0;
    rc = check_hip(hipMemcpy(&st, g->status_d, sizeof(int), hipMemcpyDeviceToHost), "status read");
    if (rc) return rc;
    if (st) {
        rc = check_hip(hipMemset(g->status_d, 0, sizeof(int)), "status clear");
        if (rc) return rc;
        return fail(HB_ERR_NONFINITE, "non-finite residual or non-positive density/pressure met");
    }
    return HB_OK;
}

}  // extern "C"
