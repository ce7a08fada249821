// Rigid grid motion for the plain FP64 kernels (ghost fill, face fluxes,
// update, loads): the per-snapshot motion table, rotation of body-frame
// vectors, the rigid grid velocity and the moving no-slip wall images.
#pragma once
#include "hb_device.hpp"

namespace hb {

// Body-frame vectors rotate by theta; the grid point whose body-frame
// position is x0 moves with theta_dot k x R(theta)(x0 - p) + (0, h_dot).
struct MotionSnap {
    double c, s, thd, h, hd;
};

__device__ __forceinline__ MotionSnap motion_snap(const Motion &mo, const BlockDesc &B, int n) {
    const double *t = mo.tab + (int64_t)kMotionW * (B.snap_off + n);
    return MotionSnap{t[0], t[1], t[2], t[3], t[4]};
}

__device__ __forceinline__ void rot2(const MotionSnap &m, double &x, double &y) {
    const double a = m.c * x - m.s * y;
    y = m.s * x + m.c * y;
    x = a;
}

__device__ __forceinline__ void grid_velocity(const MotionSnap &m, const Motion &mo, double x0,
                                              double y0, double &gx, double &gy) {
    double rx = x0 - mo.xp, ry = y0 - mo.yp;
    rot2(m, rx, ry);
    gx = -m.thd * ry;
    gy = m.thd * rx + m.hd;
}

// A ghost (i, j) of block B = blks[b] that is a no-slip wall image (j side
// wall, or the wall part of a wake cut) gets 2 u_wall added to the mirrored
// velocity, u_wall = grid velocity at the midpoint of the wall face of the
// mirrored cell's column: corner ghosts take the i-periodic partner column,
// the glued block's column across an i cut (its wall face on the same j
// side), else the nearest column.  xy: body-frame nodes of all blocks.
__device__ __forceinline__ void wall_image_motion(const BlockDesc *blks, int b, int i, int j,
                                                  const MotionSnap &m, const Motion &mo,
                                                  const double *xy, W4<double> &w) {
    const BlockDesc &B = blks[b];
    int side;
    if (j < 0) side = 2;
    else if (j >= B.nj) side = 3;
    else return;
    const int kind = B.bc[side];
    if (!(kind == HB_BC_WALL || (kind == HB_BC_WAKECUT && side == 2))) return;
    if (kind == HB_BC_WAKECUT && (i < B.wake || i >= B.ni - B.wake)) return;
    int col = i, src = b;
    if (i < 0) {
        if (B.bc[0] == HB_BC_PERIODIC) col = i + B.ni;
        else if (B.bc[0] == HB_BC_CUT) src = B.cut_blk[0], col = src < 0 ? 0 : blks[src].ni + i;
        else col = 0;
    } else if (i >= B.ni) {
        if (B.bc[1] == HB_BC_PERIODIC) col = i - B.ni;
        else if (B.bc[1] == HB_BC_CUT) src = B.cut_blk[1], col = i - B.ni;
        else col = B.ni - 1;
    }
    if (src < 0) return;          // general cuts: no moving grid (refused by hb_set_motion)
    const BlockDesc &S = blks[src];
    const int64_t nn = (int64_t)(S.ni + 1) * (S.nj + 1);
    const double *x = xy + 2 * S.node_off, *y = x + nn;
    const int64_t k = (int64_t)(side == 2 ? 0 : S.nj) * (S.ni + 1) + col;
    double gx, gy;
    grid_velocity(m, mo, 0.5 * (x[k] + x[k + 1]), 0.5 * (y[k] + y[k + 1]), gx, gy);
    w.u += 2.0 * gx;
    w.v += 2.0 * gy;
}

}  // namespace hb
