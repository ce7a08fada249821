// Grid metrics of every block, in FP64 on the device, plus FP32 copies
// rounded from the FP64 values (never computed in FP32: thin wall cells
// would lose the normal-direction differences).
//
// Layouts (per block, at the block's offsets):
//   S_I, d_I  [2][nj][ni+1]   i-face normal (dy, -dx) of the edge
//                             node(i,j)->node(i,j+1); d = centre(i,j) - centre(i-1,j)
//   S_J, d_J  [2][nj+1][ni]   j-face normal (-dy, dx) of the edge
//                             node(i,j)->node(i+1,j); d = centre(i,j) - centre(i,j-1)
//   V         [nj][ni]        cell area (half the diagonal cross product)
//   C         [2][nj][ni]     cell centre (mean of the four nodes)
// Ghost centres: periodic, wake-cut and cut ghosts are real cells (their
// centres are used); wall and far-field ghost centres are the interior
// centre mirrored across the boundary face.
#include "hb_device.hpp"

namespace hb {
namespace {

__global__ void k_cells(const BlockDesc *blks, int b, const double *xy, double *V, double *C) {
    const BlockDesc B = blks[b];
    const int64_t n = (int64_t)B.ni * B.nj;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % B.ni), j = (int)(t / B.ni);
    const int W = B.ni + 1;
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off;
    const double *y = x + nn;
    const double x1 = x[j * W + i], y1 = y[j * W + i];
    const double x2 = x[j * W + i + 1], y2 = y[j * W + i + 1];
    const double x3 = x[(j + 1) * W + i + 1], y3 = y[(j + 1) * W + i + 1];
    const double x4 = x[(j + 1) * W + i], y4 = y[(j + 1) * W + i];
    V[B.cell_off + t] = 0.5 * ((x3 - x1) * (y4 - y2) - (y3 - y1) * (x4 - x2));
    C[2 * B.cell_off + t] = 0.25 * (x1 + x2 + x3 + x4);
    C[2 * B.cell_off + n + t] = 0.25 * (y1 + y2 + y3 + y4);
}

__device__ inline void centre(const BlockDesc *blks, const double *C, int b, int i, int j,
                              double &cx, double &cy) {
    const BlockDesc &B = blks[b];
    const int64_t n = (int64_t)B.ni * B.nj;
    cx = C[2 * B.cell_off + (int64_t)j * B.ni + i];
    cy = C[2 * B.cell_off + n + (int64_t)j * B.ni + i];
}

// mirror point (px, py) across the line through a and b
__device__ inline void reflect(double px, double py, double ax, double ay, double bx, double by,
                               double &rx, double &ry) {
    const double ex = bx - ax, ey = by - ay;
    const double t = ((px - ax) * ex + (py - ay) * ey) / (ex * ex + ey * ey);
    const double fx = ax + t * ex, fy = ay + t * ey;
    rx = 2.0 * fx - px;
    ry = 2.0 * fy - py;
}

__global__ void k_faces_i(const BlockDesc *blks, int b, const double *xy, const double *C,
                          double *SI, double *dI) {
    const BlockDesc B = blks[b];
    const int W = B.ni + 1;
    const int64_t n = (int64_t)W * B.nj;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % W), j = (int)(t / W);
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off;
    const double *y = x + nn;
    const double ax = x[j * W + i], ay = y[j * W + i];
    const double bx = x[(j + 1) * W + i], by = y[(j + 1) * W + i];
    double lx, ly, rx, ry;
    if (i > 0) {
        centre(blks, C, b, i - 1, j, lx, ly);
    } else {
        double cx, cy;
        centre(blks, C, b, 0, j, cx, cy);
        if (B.bc[0] == HB_BC_PERIODIC) centre(blks, C, b, B.ni - 1, j, lx, ly);
        else if (glued_at(B, B.segs, 0, j)) {
            int a, ia, ja;
            cut_cell(blks, B.segs, b, 0, 0, j, &a, &ia, &ja);
            centre(blks, C, a, ia, ja, lx, ly);
        } else reflect(cx, cy, ax, ay, bx, by, lx, ly);
    }
    if (i < B.ni) {
        centre(blks, C, b, i, j, rx, ry);
    } else {
        double cx, cy;
        centre(blks, C, b, B.ni - 1, j, cx, cy);
        if (B.bc[1] == HB_BC_PERIODIC) centre(blks, C, b, 0, j, rx, ry);
        else if (glued_at(B, B.segs, 1, j)) {
            int a, ia, ja;
            cut_cell(blks, B.segs, b, 1, 0, j, &a, &ia, &ja);
            centre(blks, C, a, ia, ja, rx, ry);
        } else reflect(cx, cy, ax, ay, bx, by, rx, ry);
    }
    double *S = SI + 2 * B.fi_off;
    double *d = dI + 2 * B.fi_off;
    S[t] = by - ay;
    S[n + t] = -(bx - ax);
    d[t] = rx - lx;
    d[n + t] = ry - ly;
}

__global__ void k_faces_j(const BlockDesc *blks, int b, const double *xy, const double *C,
                          double *SJ, double *dJ) {
    const BlockDesc B = blks[b];
    const int W = B.ni + 1;
    const int64_t n = (int64_t)B.ni * (B.nj + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % B.ni), j = (int)(t / B.ni);
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off;
    const double *y = x + nn;
    const double ax = x[j * W + i], ay = y[j * W + i];
    const double bx = x[j * W + i + 1], by = y[j * W + i + 1];
    double lx, ly, rx, ry;
    if (j > 0) {
        centre(blks, C, b, i, j - 1, lx, ly);
    } else {
        double cx, cy;
        centre(blks, C, b, i, 0, cx, cy);
        const int kind = B.bc[2];
        const bool wake = (kind == HB_BC_WAKECUT) && (i < B.wake || i >= B.ni - B.wake);
        if (kind == HB_BC_PERIODIC) centre(blks, C, b, i, B.nj - 1, lx, ly);
        else if (wake) centre(blks, C, b, B.ni - 1 - i, 0, lx, ly);
        else if (glued_at(B, B.segs, 2, i)) {
            int a, ia, ja;
            cut_cell(blks, B.segs, b, 2, 0, i, &a, &ia, &ja);
            centre(blks, C, a, ia, ja, lx, ly);
        } else reflect(cx, cy, ax, ay, bx, by, lx, ly);
    }
    if (j < B.nj) {
        centre(blks, C, b, i, j, rx, ry);
    } else {
        double cx, cy;
        centre(blks, C, b, i, B.nj - 1, cx, cy);
        if (B.bc[3] == HB_BC_PERIODIC) centre(blks, C, b, i, 0, rx, ry);
        else if (glued_at(B, B.segs, 3, i)) {
            int a, ia, ja;
            cut_cell(blks, B.segs, b, 3, 0, i, &a, &ia, &ja);
            centre(blks, C, a, ia, ja, rx, ry);
        } else reflect(cx, cy, ax, ay, bx, by, rx, ry);
    }
    double *S = SJ + 2 * B.fj_off;
    double *d = dJ + 2 * B.fj_off;
    S[t] = -(by - ay);
    S[n + t] = bx - ax;
    d[t] = rx - lx;
    d[n + t] = ry - ly;
}

__global__ void k_round(const double *a, float *f, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) f[t] = (float)a[t];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int launch_metrics(hb_grid *g, hipStream_t s) {
    const int bs = 256;
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_cells, dim3(nblk((int64_t)B.ni * B.nj, bs)), dim3(bs), 0, s,
                           g->blk_d, b, g->xy_d, g->V_d, g->C_d);
    }
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_faces_i, dim3(nblk((int64_t)(B.ni + 1) * B.nj, bs)), dim3(bs), 0, s,
                           g->blk_d, b, g->xy_d, g->C_d, g->SI_d, g->dI_d);
        hipLaunchKernelGGL(k_faces_j, dim3(nblk((int64_t)B.ni * (B.nj + 1), bs)), dim3(bs), 0, s,
                           g->blk_d, b, g->xy_d, g->C_d, g->SJ_d, g->dJ_d);
    }
    hipLaunchKernelGGL(k_round, dim3(nblk(2 * g->n_fi, bs)), dim3(bs), 0, s, g->SI_d, g->SI_f, 2 * g->n_fi);
    hipLaunchKernelGGL(k_round, dim3(nblk(2 * g->n_fi, bs)), dim3(bs), 0, s, g->dI_d, g->dI_f, 2 * g->n_fi);
    hipLaunchKernelGGL(k_round, dim3(nblk(2 * g->n_fj, bs)), dim3(bs), 0, s, g->SJ_d, g->SJ_f, 2 * g->n_fj);
    hipLaunchKernelGGL(k_round, dim3(nblk(2 * g->n_fj, bs)), dim3(bs), 0, s, g->dJ_d, g->dJ_f, 2 * g->n_fj);
    hipLaunchKernelGGL(k_round, dim3(nblk(g->n_cells, bs)), dim3(bs), 0, s, g->V_d, g->V_f, g->n_cells);
    return check_hip(hipGetLastError(), "metrics launch");
}

}  // namespace hb
