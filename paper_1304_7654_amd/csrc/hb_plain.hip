// Plain FP64 path: one block per launch, separate kernels for ghost
// synthesis, face fluxes (both families in one launch) and the cell
// update.  Every intermediate goes through HBM.  It is the straightforward baseline that
// the fused batched kernel is measured against, and a second, independently
// structured GPU evaluation of the same residual.
#include "hb_device.hpp"
#include "hb_motion.hpp"
#include "hb_xcd.hpp"

namespace hb {
namespace {

constexpr int kBS = 256;
static_assert(kBS == kXcdBS, "one-thread-per-item kernels use 256-thread workgroups");

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

struct CellFromState {
    const BlockDesc *blks;
    const double *q;
    int n;
    double gm1;
    __device__ W4<double> operator()(int b, int i, int j) const {
        const BlockDesc &B = blks[b];
        const int64_t plane = (int64_t)B.ni * B.nj;
        const double *p = q + B.q_off + (int64_t)n * 4 * plane + (int64_t)j * B.ni + i;
        return prim_from_cons<double>(p[0], p[plane], p[2 * plane], p[3 * plane], gm1);
    }
};

struct FreeStream {
    const BlockDesc *blks;
    const double *ffw;
    int n;
    __device__ W4<double> operator()(int b) const {
        const double *f = ffw + 4 * (blks[b].snap_off + n);
        return W4<double>{f[0], f[1], f[2], f[3]};
    }
};

// Ghost-extended primitives ext[n][4][nj+4][ni+4] of one block (moving
// walls with a motion set).
__global__ void k_ghost(const BlockDesc *blks, int b, const double *q, const double *ffw,
                        double gm1, double *ext, Motion mo, const double *xy) {
    const BlockDesc &B = blks[b];
    const int we = B.ni + 4, he = B.nj + 4;
    const int64_t plane = (int64_t)we * he;
    const int64_t L = xcd_group(plane * B.ns);
    const int64_t t = L < 0 ? -1 : L * kBS + threadIdx.x;
    if (t < 0 || t >= plane * B.ns) return;
    const int n = (int)(t / plane);
    const int64_t r = t % plane;
    const int i = (int)(r % we) - 2, j = (int)(r / we) - 2;
    CellFromState cell{blks, q, n, gm1};
    FreeStream ff{blks, ffw, n};
    W4<double> w = value_ij<W4<double>>(blks, b, i, j, cell, ff, MirrorFull<double>());
    if (mo.tab) wall_image_motion(blks, b, i, j, motion_snap(mo, B, n), mo, xy, w);
    double *e = ext + B.ext_off + (int64_t)n * 4 * plane + r;
    e[0] = w.r;
    e[plane] = w.u;
    e[2 * plane] = w.v;
    e[3 * plane] = w.p;
}

__device__ inline W4<double> ld(const double *e, int64_t plane, int64_t idx) {
    return W4<double>{e[idx], e[plane + idx], e[2 * plane + idx], e[3 * plane + idx]};
}

// With a motion set, S and d of snapshot n are the body-frame ones rotated
// by theta_n, and the face moves with the grid velocity at its midpoint.
__device__ inline double moving_face(const Motion &mo, const BlockDesc &B, int n, const double *xy,
                                     int64_t kA, int64_t kB, double &sx, double &sy, double &dx,
                                     double &dy) {
    const MotionSnap m = motion_snap(mo, B, n);
    rot2(m, sx, sy);
    rot2(m, dx, dy);
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off, *y = x + nn;
    double gx, gy;
    grid_velocity(m, mo, 0.5 * (x[kA] + x[kB]), 0.5 * (y[kA] + y[kB]), gx, gy);
    return gx * sx + gy * sy;
}

__device__ __forceinline__ void flux_i(const BlockDesc *blks, int b, const double *ext,
                                       const double *SI, const double *dI, Consts c, double *FI,
                                       Motion mo, const double *xy, int64_t t) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nf = (int64_t)W * B.nj;
    if (t < 0 || t >= nf * B.ns) return;
    const int n = (int)(t / nf);
    const int64_t f = t % nf;
    const int i = (int)(f % W), j = (int)(f / W);
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    const int64_t row = (int64_t)(j + 2) * we;
    const W4<double> m2 = ld(e, plane, row + i), m1 = ld(e, plane, row + i + 1);
    const W4<double> p0 = ld(e, plane, row + i + 2), p1 = ld(e, plane, row + i + 3);
    W4<double> L, R;
    muscl(m2, m1, p0, p1, c.eps, L, R);
    double sx = SI[2 * B.fi_off + f], sy = SI[2 * B.fi_off + nf + f];
    double dx = dI[2 * B.fi_off + f], dy = dI[2 * B.fi_off + nf + f];
    double vg = 0.0;
    if (mo.tab) vg = moving_face(mo, B, n, xy, (int64_t)j * W + i, (int64_t)(j + 1) * W + i, sx, sy, dx, dy);
    double fl[4];
    roe_flux(L, R, sx, sy, c.gamma, c.delta_frac, fl, vg);
    // viscous: L = cell (i-1, j), R = cell (i, j); edge from node (i, j) to (i, j+1)
    const double g = c.gamma;
    const UVT<double> uL = uvt(m1, g), uR = uvt(p0, g);
    const int64_t lo = (int64_t)(j + 1) * we, hi = (int64_t)(j + 3) * we;
    const UVT<double> nA = avg4(uvt(ld(e, plane, lo + i + 1), g), uvt(ld(e, plane, lo + i + 2), g),
                                uL, uR);
    const UVT<double> nB = avg4(uL, uR, uvt(ld(e, plane, hi + i + 1), g),
                                uvt(ld(e, plane, hi + i + 2), g));
    double fv[3];
    viscous_flux(uL, uR, nA, nB, sx, sy, dx, dy, c.mu, c.kappa, fv);
    double *o = FI + B.fiq_off + (int64_t)n * 4 * nf + f;
    o[0] = fl[0];
    o[nf] = fl[1] - fv[0];
    o[2 * nf] = fl[2] - fv[1];
    o[3 * nf] = fl[3] - fv[2];
}

__device__ __forceinline__ void flux_j(const BlockDesc *blks, int b, const double *ext,
                                       const double *SJ, const double *dJ, Consts c, double *FJ,
                                       Motion mo, const double *xy, int64_t t) {
    const BlockDesc &B = blks[b];
    const int64_t nf = (int64_t)B.ni * (B.nj + 1);
    if (t < 0 || t >= nf * B.ns) return;
    const int n = (int)(t / nf);
    const int64_t f = t % nf;
    const int i = (int)(f % B.ni), j = (int)(f / B.ni);
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    const int col = i + 2;
    const W4<double> m2 = ld(e, plane, (int64_t)j * we + col);
    const W4<double> m1 = ld(e, plane, (int64_t)(j + 1) * we + col);
    const W4<double> p0 = ld(e, plane, (int64_t)(j + 2) * we + col);
    const W4<double> p1 = ld(e, plane, (int64_t)(j + 3) * we + col);
    W4<double> L, R;
    muscl(m2, m1, p0, p1, c.eps, L, R);
    double sx = SJ[2 * B.fj_off + f], sy = SJ[2 * B.fj_off + nf + f];
    double dx = dJ[2 * B.fj_off + f], dy = dJ[2 * B.fj_off + nf + f];
    double vg = 0.0;
    if (mo.tab) {
        const int64_t kA = (int64_t)j * (B.ni + 1) + i;
        vg = moving_face(mo, B, n, xy, kA, kA + 1, sx, sy, dx, dy);
    }
    double fl[4];
    roe_flux(L, R, sx, sy, c.gamma, c.delta_frac, fl, vg);
    // viscous: L = cell (i, j-1), R = cell (i, j); edge from node (i+1, j) to (i, j)
    const double g = c.gamma;
    const UVT<double> uL = uvt(m1, g), uR = uvt(p0, g);
    const int64_t r1 = (int64_t)(j + 1) * we, r2 = (int64_t)(j + 2) * we;
    const UVT<double> nA = avg4(uvt(ld(e, plane, r1 + col - 1), g), uL,
                                uvt(ld(e, plane, r2 + col - 1), g), uR);          // node (i, j)
    const UVT<double> nB = avg4(uL, uvt(ld(e, plane, r1 + col + 1), g), uR,
                                uvt(ld(e, plane, r2 + col + 1), g));              // node (i+1, j)
    double fv[3];
    viscous_flux(uL, uR, nB, nA, sx, sy, dx, dy, c.mu, c.kappa, fv);
    double *o = FJ + B.fjq_off + (int64_t)n * 4 * nf + f;
    o[0] = fl[0];
    o[nf] = fl[1] - fv[0];
    o[2 * nf] = fl[2] - fv[1];
    o[3 * nf] = fl[3] - fv[2];
}

// Both face families of block b in one launch: items [0, nI) are the
// i-faces of all snapshots, the rest the j-faces.
__global__ void __launch_bounds__(kBS) k_flux(const BlockDesc *blks, int b, const double *ext,
                                              const double *SI, const double *dI, const double *SJ,
                                              const double *dJ, Consts c, double *FI, double *FJ,
                                              Motion mo, const double *xy, int64_t nI, int64_t nJ) {
    const int64_t lw = xcd_group(nI + nJ);
    if (lw < 0) return;
    const int64_t t = lw * kBS + threadIdx.x;
    if (t < nI) flux_i(blks, b, ext, SI, dI, c, FI, mo, xy, t);
    else flux_j(blks, b, ext, SJ, dJ, c, FJ, mo, xy, t - nI);
}

// Cell update, one thread per cell and snapshot.  mode 0: out = R*(qin).
// mode 1: out = q0 - alpha (dtau/V) R*(qin), dtau from q0; with `norm` set,
// each workgroup's partial sum of (R*_rho/V)^2 goes to
// partials[part_off + logical workgroup].  Logical workgroup L takes
// snapshot L mod N_s of the cell group L / N_s (256 cells), so the N_s
// workgroups that read the same cells for the HB source are neighbours (one
// XCD, one L2); each thread reads its cell's stage input of every snapshot
// into registers.
__global__ void __launch_bounds__(kBS) k_update(const BlockDesc *blks, int b, const double *FI,
                                               const double *FJ, const double *SI, const double *SJ,
                                               const double *V, const double *D, const double *qin,
                                               const double *q0, double *out, int mode, double alpha,
                                               int norm, double *partials, int *status, Consts c,
                                               Motion mo, const double *C) {
    const BlockDesc &B = blks[b];
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int64_t L = xcd_group(((plane + kBS - 1) / kBS) * B.ns * kBS);
    if (L < 0) return;                     // a whole padding workgroup
    const int n = (int)(L % B.ns);
    const int64_t t = (L / B.ns) * kBS + threadIdx.x;
    double acc = 0.0;
    int bad = 0;
    if (t < plane) {
        const int i = (int)(t % B.ni), j = (int)(t / B.ni);
        const int W = B.ni + 1;
        const int64_t nfi = (int64_t)W * B.nj, nfj = (int64_t)B.ni * (B.nj + 1);
        const int64_t fi0 = (int64_t)j * W + i, fj0 = t;
        const double vol = V[B.cell_off + t];
        const double *dm = D + B.d_off + n * kNsPad;
        const double *qi = qin + B.q_off + t;
        double qm[kMaxNs][4];
#pragma unroll
        for (int m = 0; m < kMaxNs; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) qm[m][v] = m < B.ns ? qi[((int64_t)m * 4 + v) * plane] : 0.0;
        double rs[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double *fi = FI + B.fiq_off + ((int64_t)n * 4 + v) * nfi;
            const double *fj = FJ + B.fjq_off + ((int64_t)n * 4 + v) * nfj;
            double src = 0.0;
#pragma unroll
            for (int m = 0; m < kMaxNs; ++m)
                if (m < B.ns) src += dm[m] * qm[m][v];
            rs[v] = (fi[fi0 + 1] - fi[fi0]) + (fj[fj0 + B.ni] - fj[fj0]) + vol * src;
        }
        const int64_t o = B.q_off + (int64_t)n * 4 * plane + t;
        if (mode == 0) {
            for (int v = 0; v < 4; ++v) out[o + v * plane] = rs[v];
        } else {
            const double *b0 = q0 + o;
            W4<double> w0 = prim_from_cons<double>(b0[0], b0[plane], b0[2 * plane], b0[3 * plane],
                                                   c.gamma - 1.0);
            double ax = 0.5 * (SI[2 * B.fi_off + fi0] + SI[2 * B.fi_off + fi0 + 1]);
            double ay = 0.5 * (SI[2 * B.fi_off + nfi + fi0] + SI[2 * B.fi_off + nfi + fi0 + 1]);
            double bx = 0.5 * (SJ[2 * B.fj_off + fj0] + SJ[2 * B.fj_off + fj0 + B.ni]);
            double by = 0.5 * (SJ[2 * B.fj_off + nfj + fj0] + SJ[2 * B.fj_off + nfj + fj0 + B.ni]);
            if (mo.tab) {   // snapshot's normals, velocity relative to the grid at the centre
                const MotionSnap m = motion_snap(mo, B, n);
                rot2(m, ax, ay);
                rot2(m, bx, by);
                double gx, gy;
                grid_velocity(m, mo, C[2 * B.cell_off + t], C[2 * B.cell_off + plane + t], gx, gy);
                w0.u -= gx;
                w0.v -= gy;
            }
            const double dt = local_dt<double>(w0, ax, ay, bx, by, vol, c.gamma, c.mu / c.prandtl,
                                               c.cfl, B.omega_nh);
            const double fac = alpha * dt / vol;
            double nq[4];
            for (int v = 0; v < 4; ++v) nq[v] = b0[v * plane] - fac * rs[v];
            for (int v = 0; v < 4; ++v) out[o + v * plane] = nq[v];
            const double pn = (c.gamma - 1.0) * (nq[3] - 0.5 * (nq[1] * nq[1] + nq[2] * nq[2]) / nq[0]);
            if (!(nq[0] > 0.0) || !(pn > 0.0) || !isfinite(rs[0] + rs[1] + rs[2] + rs[3])) bad = 1;
        }
        const double rr = rs[0] / vol;
        acc = rr * rr;
    }
    // one atomic per wave that met a bad cell
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, 1);
    if (!norm) return;
    __shared__ double red[kBS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[B.part_off + L] = red[0];
}

Metrics<double> fp64_metrics(hb_grid *g) {
    return Metrics<double>{g->SI_d, g->dI_d, g->SJ_d, g->dJ_d, g->V_d};
}

// Side streams and their events, created on first use.
int side_streams(hb_grid *g) {
    if (g->fork_ev) return HB_OK;
    for (int k = 0; k < hb_grid::kSide; ++k) {
        int rc = check_hip(hipStreamCreateWithFlags(&g->side[k], hipStreamNonBlocking), "side stream");
        rc = rc ? rc : check_hip(hipEventCreateWithFlags(&g->join_ev[k], hipEventDisableTiming), "event");
        if (rc) return rc;
    }
    return check_hip(hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming), "event");
}

// One stage over all blocks.  A block's four kernels only write its own
// regions of the ghost-extended field, the face fluxes and `out`, and read
// the stage input `qin` (also the glued blocks' cells) and `q0`, which no
// kernel of the stage writes (`out` may be `q0` itself, read and written
// pointwise by the block's own update).  So the blocks run on side streams
// (block b on stream b mod kSide; 8 measured faster than 4, 12 or 16 on a
// 32-block batch), forked from and joined back to `s`.
int stage(hb_grid *g, const double *qin, const double *q0, double *out, int mode, double alpha,
          int norm, hipStream_t s) {
    const Consts c = g->consts;
    const bool fork = g->nblocks > 1;
    if (fork) {
        int rc = side_streams(g);
        rc = rc ? rc : check_hip(hipEventRecord(g->fork_ev, s), "fork");
        for (int k = 0; k < hb_grid::kSide && !rc; ++k)
            rc = check_hip(hipStreamWaitEvent(g->side[k], g->fork_ev, 0), "fork");
        if (rc) return rc;
    }
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipStream_t st = fork ? g->side[b % hb_grid::kSide] : s;
        const int64_t next = (int64_t)(B.ni + 4) * (B.nj + 4) * B.ns;
        hipLaunchKernelGGL(k_ghost, dim3(xcd_grid(next)), dim3(kBS), 0, st, g->blk_d, b, qin, g->ffw_d,
                           c.gamma - 1.0, g->ext_d, g->motion, g->xy_d);
        const int64_t nI = (int64_t)(B.ni + 1) * B.nj * B.ns, nJ = (int64_t)B.ni * (B.nj + 1) * B.ns;
        hipLaunchKernelGGL(k_flux, dim3(xcd_grid(nI + nJ)), dim3(kBS), 0, st, g->blk_d, b, g->ext_d,
                           g->SI_d, g->dI_d, g->SJ_d, g->dJ_d, c, g->FI_d, g->FJ_d, g->motion, g->xy_d,
                           nI, nJ);
        hipLaunchKernelGGL(k_update, dim3(xcd_grid((int64_t)nblk((int64_t)B.ni * B.nj) * B.ns * kBS)),
                           dim3(kBS), 0, st, g->blk_d, b,
                           g->FI_d, g->FJ_d, g->SI_d, g->SJ_d, g->V_d, g->D_d, qin, q0, out, mode,
                           alpha, norm, g->partials_d, g->status_d, c, g->motion, g->C_d);
    }
    int rc = check_hip(hipGetLastError(), "plain stage launch");
    for (int k = 0; fork && k < hb_grid::kSide && !rc; ++k) {
        rc = check_hip(hipEventRecord(g->join_ev[k], g->side[k]), "join");
        rc = rc ? rc : check_hip(hipStreamWaitEvent(s, g->join_ev[k], 0), "join");
    }
    return rc;
}

}  // namespace

// Ghost-extended primitives of block b (also used by the adjoint).
int plain_ghost_fill(hb_grid *g, int b, const double *q, double *ext, hipStream_t s) {
    const BlockDesc &B = g->blk[b];
    const int64_t next = (int64_t)(B.ni + 4) * (B.nj + 4) * B.ns;
    hipLaunchKernelGGL(k_ghost, dim3(xcd_grid(next)), dim3(kBS), 0, s, g->blk_d, b, q, g->ffw_d,
                       g->consts.gamma - 1.0, ext, g->motion, g->xy_d);
    return check_hip(hipGetLastError(), "ghost launch");
}

// Number of norm partials the plain path writes for a block.
int64_t plain_partials(const BlockDesc &B) { return (int64_t)nblk((int64_t)B.ni * B.nj) * B.ns; }

int plain_residual(hb_grid *g, const double *q, double *r, hipStream_t s) {
    return stage(g, q, q, r, 0, 0.0, 0, s);
}

int plain_rk_iterate(hb_grid *g, double *q, int n_iter, double *resnorm, hipStream_t s) {
    const int ns = g->solver.n_stages;
    int rc = launch_reset_ctr(g->ctr_d, s);
    if (rc) return rc;
    for (int it = 0; it < n_iter; ++it) {
        const double *in = q;
        for (int k = 0; k < ns; ++k) {
            // the last stage writes q in place (q is read pointwise only);
            // a one-stage scheme reads q as its stencil input, so it goes
            // through a scratch buffer
            double *out = (k == ns - 1 && ns > 1) ? q : ((k % 2 == 0) ? g->qa_d : g->qb_d);
            hipEvent_t end;
            rc = prof_begin(g, s, &end);
            if (rc) return rc;
            rc = stage(g, in, q, out, 1, g->solver.rk_alpha[k], k == 0, s);
            if (rc) return rc;
            rc = prof_end(end, s);
            if (rc) return rc;
            in = out;
        }
        if (ns == 1) {
            rc = check_hip(hipMemcpyAsync(q, g->qa_d, sizeof(double) * g->n_state,
                                          hipMemcpyDeviceToDevice, s), "copy");
            if (rc) return rc;
        }
        rc = launch_norm_finalize(g, g->partials_d, g->n_partials, resnorm, g->ctr_d, s);
        if (rc) return rc;
    }
    return HB_OK;
}

}  // namespace hb
