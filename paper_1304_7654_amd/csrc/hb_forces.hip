// Force coefficients per body and snapshot, FP64 (the paper's
// cl(n, ibody), cd(n, ibody), cm(n, ibody) and their single aggregated
// reduction per Runge-Kutta step, §MPI Optimisations).  One workgroup per
// (block, snapshot) sums its wall faces in a fixed order; a second kernel
// adds the blocks of each body in block order and rotates to wind axes.
// No atomics: results are bitwise reproducible.
#include "hb_device.hpp"
#include "hb_motion.hpp"

namespace hb {
namespace {

constexpr int kBS = 256;

struct CellQ {
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

struct FF {
    const BlockDesc *blks;
    const double *ffw;
    int n;
    __device__ W4<double> operator()(int b) const {
        const double *f = ffw + 4 * (blks[b].snap_off + n);
        return W4<double>{f[0], f[1], f[2], f[3]};
    }
};

// Loads of one jmin wall face: (Fx, Fy, Mz).
__device__ inline void face_load(const BlockDesc *blks, int b, int n, int i, const double *q,
                                 const double *ffw, const double *xy, const double *SJ,
                                 const double *dJ, const Consts &c, double xm, double ym,
                                 const Motion &mo, double out[3]) {
    const BlockDesc &B = blks[b];
    CellQ cell{blks, q, n, c.gamma - 1.0};
    FF ff{blks, ffw, n};
    const double g = c.gamma;
    MotionSnap ms{1.0, 0.0, 0.0, 0.0, 0.0};
    if (mo.tab) ms = motion_snap(mo, B, n);
    // (i', j') resolved like every ghost, moving-wall images with a motion set
    auto val = [&](int ii, int jj) {
        W4<double> w = value_ij<W4<double>>(blks, b, ii, jj, cell, ff, MirrorFull<double>());
        if (mo.tab) wall_image_motion(blks, b, ii, jj, ms, mo, xy, w);
        return w;
    };
    const W4<double> wR = val(i, 0);
    const W4<double> wL = val(i, -1);
    const UVT<double> uL = uvt(wL, g), uR = uvt(wR, g);
    const UVT<double> nA = avg4(uvt(val(i - 1, -1), g), uL, uvt(val(i - 1, 0), g), uR);
    const UVT<double> nB = avg4(uL, uvt(val(i + 1, -1), g), uR, uvt(val(i + 1, 0), g));
    const int64_t nf = (int64_t)B.ni * (B.nj + 1);
    double sx = SJ[2 * B.fj_off + i], sy = SJ[2 * B.fj_off + nf + i];
    double dx = dJ[2 * B.fj_off + i], dy = dJ[2 * B.fj_off + nf + i];
    if (mo.tab) {   // the snapshot's grid: body-frame vectors rotated by theta_n
        rot2(ms, sx, sy);
        rot2(ms, dx, dy);
    }
    double fv[3];
    viscous_flux(uL, uR, nB, nA, sx, sy, dx, dy, c.mu, c.kappa, fv);
    const double dp = wR.p - c.pinf;
    const double fx = -dp * sx + fv[0];
    const double fy = -dp * sy + fv[1];
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off;
    const double *y = x + nn;
    // moment arm: a body-frame difference, rotated with the body
    double mx = 0.5 * (x[i] + x[i + 1]) - xm;
    double my = 0.5 * (y[i] + y[i + 1]) - ym;
    if (mo.tab) rot2(ms, mx, my);
    out[0] = fx;
    out[1] = fy;
    out[2] = mx * fy - my * fx;
}

// Workgroup (block b, snapshot n, chunk k): the wall faces i = 256 k + tid,
// one per thread; the chunk's sum goes to part[((b kMaxNs + n) nch + k)].
__global__ void k_block_loads(const BlockDesc *blks, const double *q, const double *ffw,
                              const double *xy, const double *SJ, const double *dJ, Consts c,
                              double xm, double ym, Motion mo, int nch, double *part) {
    const int b = blockIdx.x;
    const int n = blockIdx.y;
    const int i = blockIdx.z * kBS + threadIdx.x;
    const BlockDesc &B = blks[b];
    double acc[3] = {0.0, 0.0, 0.0};
    if (n < B.ns && i < B.ni && jmin_wall(B, i))
        face_load(blks, b, n, i, q, ffw, xy, SJ, dJ, c, xm, ym, mo, acc);
    __shared__ double red[3][kBS];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && n < B.ns)
        for (int k = 0; k < 3; ++k)
            part[(((int64_t)b * kMaxNs + n) * nch + blockIdx.z) * 3 + k] = red[k][0];
}

// One thread per (body, snapshot) entry of the output; the blocks of a body
// (body_blk[body_ptr[body] ..], in block order) are summed in block order.
__global__ void k_body_coeffs(const int *body_ptr, const int *body_blk, const int *body_off,
                              const int *body_ns, int nbody, const double *part, int nch,
                              double ca, double sa, double qinf_l, double qinf_l2, double *cf) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int body = 0, n = t;
    while (body < nbody && n >= body_ns[body]) {
        n -= body_ns[body];
        ++body;
    }
    if (body >= nbody) return;
    double fx = 0.0, fy = 0.0, mz = 0.0;
    for (int k = body_ptr[body]; k < body_ptr[body + 1]; ++k) {
        const double *p = part + ((int64_t)body_blk[k] * kMaxNs + n) * nch * 3;
        for (int h = 0; h < nch; ++h) {
            fx += p[3 * h];
            fy += p[3 * h + 1];
            mz += p[3 * h + 2];
        }
    }
    double *o = cf + body_off[body] + 3 * n;
    o[0] = (-fx * sa + fy * ca) / qinf_l;
    o[1] = (fx * ca + fy * sa) / qinf_l;
    o[2] = -mz / qinf_l2;
}

}  // namespace

int launch_forces(hb_grid *g, const double *q, double *cf, hipStream_t s) {
    hipLaunchKernelGGL(k_block_loads, dim3(g->nblocks, kMaxNs, g->fchunks), dim3(kBS), 0, s, g->blk_d,
                       q, g->ffw_d, g->xy_d, g->SJ_d, g->dJ_d, g->consts, g->flow.x_mom,
                       g->flow.y_mom, g->motion, g->fchunks, g->fpart_d);
    const int total = (int)(g->n_forces / 3);
    const double qinf = 0.5 * g->flow.mach * g->flow.mach;
    const double L = g->flow.l_ref;
    hipLaunchKernelGGL(k_body_coeffs, dim3((total + 63) / 64), dim3(64), 0, s, g->body_ptr_d,
                       g->body_blk_d, g->body_off_d, g->body_ns_d, g->nbody, g->fpart_d, g->fchunks,
                       cos(g->flow.alpha0), sin(g->flow.alpha0), qinf * L, qinf * L * L, cf);
    return check_hip(hipGetLastError(), "forces launch");
}

}  // namespace hb
