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

// A ghost (i, j) of block b that is a no-slip wall image takes the grid
// velocity at the midpoint of the wall face at which its resolution
// (value_ij) mirrors: for a corner ghost that is the column its i-side rule
// led to (the i-periodic partner column, the glued block's column across
// an i cut).  Returns false for a ghost that is no wall image; else *src =
// the block holding the wall face and *k = the index of its first node
// (the second is k + 1).  Walls lie on j sides only (hb_set_motion refuses
// others), so a ghost meets at most one.
struct WallSeen {
    int *b, *side, *pos;
    __device__ void operator()(int bb, int s, int p) const {
        *b = bb;
        *side = s;
        *pos = p;
    }
};
struct NoValue {
    __device__ int operator()(int, int, int) const { return 0; }
    __device__ int operator()(int) const { return 0; }
};

__device__ __forceinline__ bool wall_image_face(const BlockDesc *blks, int b, int i, int j, int *src,
                                                int64_t *k) {
    int wb = -1, ws = 0, wp = 0;
    const NoValue none;
    value_ij<int>(blks, b, i, j, none, none, [](int x) { return x; }, WallSeen{&wb, &ws, &wp});
    if (wb < 0 || ws < 2) return false;
    const BlockDesc &S = blks[wb];
    *src = wb;
    *k = (int64_t)(ws == 2 ? 0 : S.nj) * (S.ni + 1) + wp;
    return true;
}

// The moving-wall image u_g = 2 u_wall - u: adds 2 u_wall to the mirrored
// velocity of ghost (i, j).  xy: body-frame nodes of all blocks.
__device__ __forceinline__ void wall_image_motion(const BlockDesc *blks, int b, int i, int j,
                                                  const MotionSnap &m, const Motion &mo,
                                                  const double *xy, W4<double> &w) {
    int s;
    int64_t k;
    if (!wall_image_face(blks, b, i, j, &s, &k)) return;
    const BlockDesc &S = blks[s];
    const int64_t nn = (int64_t)(S.ni + 1) * (S.nj + 1);
    const double *x = xy + 2 * S.node_off, *y = x + nn;
    double gx, gy;
    grid_velocity(m, mo, 0.5 * (x[k] + x[k + 1]), 0.5 * (y[k] + y[k + 1]), gx, gy);
    w.u += 2.0 * gx;
    w.v += 2.0 * gy;
}

// Adjoint of the rigid grid velocity at a body-frame point with respect to
// that point: (gx, gy) = theta_dot (-r_y, r_x) + (0, h_dot), r = R (x0 - p),
// so x0bar = theta_dot R^T (gybar, -gxbar).
__device__ __forceinline__ void grid_velocity_rev(const MotionSnap &m, double gxb, double gyb,
                                                  double &xb, double &yb) {
    const double rx = m.thd * gyb, ry = -m.thd * gxb;
    xb = m.c * rx + m.s * ry;
    yb = -m.s * rx + m.c * ry;
}

// R^T v: a rotated vector's adjoint taken back to the body frame.
__device__ __forceinline__ void rot2_rev(const MotionSnap &m, double &x, double &y) {
    const double a = m.c * x + m.s * y;
    y = -m.s * x + m.c * y;
    x = a;
}

}  // namespace hb
