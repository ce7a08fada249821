// Reverse mode of the HB residual (FP64): products with the transposed
// Jacobians of R* with respect to the state, the node coordinates and the
// mean incidence.  Nothing from the forward evaluation is stored: each face
// recomputes its reconstruction, Roe and viscous fluxes from the state.
//
// Steps (one block per launch, all snapshots):
//  1. ghost-extended primitives of q (the plain path's ghost kernel);
//  2. face kernels: the adjoint of each face flux is rbar(L) - rbar(R); the
//     reverse sweep through Roe, MUSCL and the viscous flux gives adjoint
//     terms for the face's four line cells, its two edge nodes, its normal S
//     and its centre offset d, stored per face (kAF doubles);
//  3. node gather: each node sums the (u, v, T) adjoints of the faces
//     that use it;
//  4. cell gather over the ghost-extended index range: each cell sums the
//     terms of the faces whose stencils contain it and a quarter of each of
//     its four nodes (converted to primitives);
//  5. fold: each interior cell adds the adjoints of the ghost cells that
//     copy it (periodic, wake cut, wall mirror, block cut; a host-built
//     inverse of the ghost rules, so no atomics), converts to conserved
//     variables and adds the HB source term V D^T rbar;
//  6. far-field ghosts carry the incidence: their adjoints reduce to the
//     alpha0 derivative (one partial per workgroup, summed in a fixed order);
//  7. node coordinates: the metric adjoints (S, d per face; V per cell, taken
//     in the fold) are chained to the nodes with FP64 atomic adds (summation
//     order, hence the last bits of xybar, may vary from run to run).
//
// The force coefficients are a functional of the wall faces only (jmin,
// j = 0): the adjoint of the wall-cell pressure, of the wall-face viscous
// flux and of the face normal are written into the same per-face records
// (all other records are zero), the face-midpoint moment arms go to the
// nodes directly, and steps 3-7 run unchanged without the HB source and cell
// area terms.  The incidence also enters through the wind axes:
// d cd / d alpha0 = cl and d cl / d alpha0 = -cd.
#include "hb_device.hpp"
#include "hb_motion.hpp"
#include "hb_xcd.hpp"

#include <vector>

namespace hb {

int plain_ghost_fill(hb_grid *g, int b, const double *q, double *ext, hipStream_t s);

namespace {

constexpr int kBS = 256;
static_assert(kBS == kXcdBS, "one-thread-per-item kernels use 256-thread workgroups");
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// forward pieces recomputed by the reverse sweeps, with adj_rcp in place of
// the exact division: (u, v, T = gamma p / rho) of a primitive state and
// the MUSCL / van Albada face states
__device__ __forceinline__ UVT<double> uvt_a(const W4<double> &w, double g) {
    return UVT<double>{w.u, w.v, g * w.p * adj_rcp(w.r)};
}
__device__ __forceinline__ double va_a(double a, double b, double eps) {
    return (a + b) * (a * b + eps) * adj_rcp(a * a + b * b + 2.0 * eps);
}
__device__ __forceinline__ void muscl_a(const W4<double> &m2, const W4<double> &m1, const W4<double> &p0,
                                        const W4<double> &p1, double eps, W4<double> &L, W4<double> &R) {
    L.r = m1.r + 0.5 * va_a(m1.r - m2.r, p0.r - m1.r, eps);
    L.u = m1.u + 0.5 * va_a(m1.u - m2.u, p0.u - m1.u, eps);
    L.v = m1.v + 0.5 * va_a(m1.v - m2.v, p0.v - m1.v, eps);
    L.p = m1.p + 0.5 * va_a(m1.p - m2.p, p0.p - m1.p, eps);
    R.r = p0.r - 0.5 * va_a(p0.r - m1.r, p1.r - p0.r, eps);
    R.u = p0.u - 0.5 * va_a(p0.u - m1.u, p1.u - p0.u, eps);
    R.v = p0.v - 0.5 * va_a(p0.v - m1.v, p1.v - p0.v, eps);
    R.p = p0.p - 0.5 * va_a(p0.p - m1.p, p1.p - p0.p, eps);
}

// Per-face records are written once and read once by the gathers.  When a
// block's records outgrow the 256 MB last-level cache they are stored
// non-temporally, so that they do not evict the face kernel's inputs
// (1024x512, N_H = 4: adjoint 1.51 -> 1.46 ms); smaller blocks store them
// normally and the gathers find them in the cache (non-temporal stores at
// 256x128, N_H = 2, measured 2% slower).
template <bool NT>
__device__ __forceinline__ void ntst(double *p, double v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ inline W4<double> ldw(const double *e, int64_t plane, int64_t idx) {
    return W4<double>{e[idx], e[plane + idx], e[2 * plane + idx], e[3 * plane + idx]};
}

// r_bar of interior cell (i, j) of snapshot n, all 4 variables (0 outside)
__device__ inline void rbar_cell(const BlockDesc &B, const double *rbar, int n, int i, int j,
                                 double out[4]) {
    if (i < 0 || i >= B.ni || j < 0 || j >= B.nj) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    const int64_t plane = (int64_t)B.ni * B.nj;
    const double *r = rbar + B.q_off + (int64_t)n * 4 * plane + (int64_t)j * B.ni + i;
    out[0] = r[0];
    out[1] = r[plane];
    out[2] = r[2 * plane];
    out[3] = r[3 * plane];
}

// Reverse sweep of one face.  Line cells m2, m1, p0, p1 (ext indices x0..x3),
// node values at the edge start P and end Q.  Fb: adjoint of the net face
// flux.  Writes the kAF adjoint terms to out[k * nf] (k = component).
template <bool NT, bool MV, bool GEO>
__device__ inline void face_rev(const double *e, int64_t plane, const int x[4], const UVT<double> &P,
                                const UVT<double> &Q, double sx, double sy, double dx, double dy,
                                const double Fb[4], const Consts &c, double *out, int64_t nf,
                                double vg, const MotionSnap *ms, double gx, double gy, double *mb,
                                int64_t mbs) {
    const double g = c.gamma;
    // viscous part first (net flux = Roe - viscous: it sees -Fb, its mass
    // term is 0): its node adjoints are final at once and are stored, which
    // keeps fewer values live across the Roe reverse
    double sxb = 0.0, syb = 0.0, dxb = 0.0, dyb = 0.0;
    UVT<double> uLb{0, 0, 0}, uRb{0, 0, 0};
    {
        const double fvb[3] = {-Fb[1], -Fb[2], -Fb[3]};
        const UVT<double> uL = uvt_a(ldw(e, plane, x[1]), g), uR = uvt_a(ldw(e, plane, x[2]), g);
        UVT<double> Pb{0, 0, 0}, Qb{0, 0, 0};
        viscous_flux_rev(uL, uR, P, Q, sx, sy, dx, dy, c.mu, c.kappa, fvb, uLb, uRb, Pb, Qb, sxb, syb,
                         dxb, dyb);
        ntst<NT>(out + 16 * nf, Pb.u);
        ntst<NT>(out + 17 * nf, Pb.v);
        ntst<NT>(out + 18 * nf, Pb.t);
        ntst<NT>(out + 19 * nf, Qb.u);
        ntst<NT>(out + 20 * nf, Qb.v);
        ntst<NT>(out + 21 * nf, Qb.t);
    }
    W4<double> Lb{0, 0, 0, 0}, Rb{0, 0, 0, 0};
    {
        const W4<double> m2 = ldw(e, plane, x[0]), m1 = ldw(e, plane, x[1]);
        const W4<double> p0 = ldw(e, plane, x[2]), p1 = ldw(e, plane, x[3]);
        W4<double> L, R;
        muscl_a(m2, m1, p0, p1, c.eps, L, R);
        double vgb = 0.0;
        roe_flux_rev(L, R, sx, sy, g, c.delta_frac, Fb, Lb, Rb, sxb, syb, vg, MV ? &vgb : nullptr);
        if constexpr (MV) {
            // vg = (gx, gy) . S, (gx, gy) the grid velocity at the body-frame
            // midpoint; S and d are the body-frame vectors rotated by theta_n
            sxb += vgb * gx;
            syb += vgb * gy;
            if (mb) {
                double xb, yb;
                grid_velocity_rev(*ms, vgb * sx, vgb * sy, xb, yb);
                mb[0] = xb;
                mb[mbs] = yb;
            }
            rot2_rev(*ms, sxb, syb);
            rot2_rev(*ms, dxb, dyb);
        }
    }
    if constexpr (GEO) {        // read only by the coordinate adjoints
        ntst<NT>(out + 22 * nf, sxb);
        ntst<NT>(out + 23 * nf, syb);
        ntst<NT>(out + 24 * nf, dxb);
        ntst<NT>(out + 25 * nf, dyb);
    }
    const W4<double> m2 = ldw(e, plane, x[0]), m1 = ldw(e, plane, x[1]);
    const W4<double> p0 = ldw(e, plane, x[2]), p1 = ldw(e, plane, x[3]);
    double cb[4][4] = {{0}};
    const double Lv[4] = {Lb.r, Lb.u, Lb.v, Lb.p}, Rv[4] = {Rb.r, Rb.u, Rb.v, Rb.p};
    const double M2[4] = {m2.r, m2.u, m2.v, m2.p}, M1[4] = {m1.r, m1.u, m1.v, m1.p};
    const double P0[4] = {p0.r, p0.u, p0.v, p0.p}, P1[4] = {p1.r, p1.u, p1.v, p1.p};
    for (int v = 0; v < 4; ++v)
        muscl_rev1(M2[v], M1[v], P0[v], P1[v], c.eps, Lv[v], Rv[v], cb[0][v], cb[1][v], cb[2][v],
                   cb[3][v]);
    W4<double> w1{cb[1][0], cb[1][1], cb[1][2], cb[1][3]};
    uvt_rev(m1, uLb, g, w1);
    W4<double> w2{cb[2][0], cb[2][1], cb[2][2], cb[2][3]};
    uvt_rev(p0, uRb, g, w2);
    cb[1][0] = w1.r; cb[1][1] = w1.u; cb[1][2] = w1.v; cb[1][3] = w1.p;
    cb[2][0] = w2.r; cb[2][1] = w2.u; cb[2][2] = w2.v; cb[2][3] = w2.p;
    for (int r = 0; r < 4; ++r)
        for (int v = 0; v < 4; ++v) ntst<NT>(out + (r * 4 + v) * nf, cb[r][v]);
}

// Node slots: i-faces store node (i, j) [edge start] in slot 0 (components
// 16..18) and node (i, j+1) [end] in slot 1 (19..21); j-faces store node
// (i+1, j) [start] in slot 0 and node (i, j) [end] in slot 1.
// On a moving grid (mo.tab) the face's S and d are those of snapshot n (the
// body-frame vectors rotated by theta_n) and it moves with the grid velocity
// (gx, gy) at its midpoint (the forward flux of the plain kernels): returns
// vg = (gx, gy) . S.  The face kernels then store the S and d adjoints taken
// back to the body frame, and, with Mb, the adjoint of the body-frame
// midpoint per face and snapshot ([2][nf] per snapshot, offsets afi_off /
// kAF * 2 and afj_off / kAF * 2).
__device__ __forceinline__ double moving_geo(const Motion &mo, const BlockDesc &B, int n, const double *xy,
                                             int64_t kA, int64_t kB, double &sx, double &sy, double &dx,
                                             double &dy, MotionSnap &m, double &gx, double &gy) {
    m = motion_snap(mo, B, n);
    rot2(m, sx, sy);
    rot2(m, dx, dy);
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off, *y = x + nn;
    grid_velocity(m, mo, 0.5 * (x[kA] + x[kB]), 0.5 * (y[kA] + y[kB]), gx, gy);
    return gx * sx + gy * sy;
}

template <bool NT, bool MV, bool GEO>
__device__ __forceinline__ void adj_face_i(const BlockDesc *blks, int b, const double *ext, const double *SI,
                             const double *dI, const double *rbar, Consts c, double *AF, Motion mo,
                             const double *xy, double *Mb, int64_t tid_) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nf = (int64_t)W * B.nj;
    const int64_t t = tid_;
    if (t >= nf * B.ns) return;
    const int n = (int)(t / nf);
    const int64_t f = t % nf;
    const int i = (int)(f % W), j = (int)(f / W);
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    const int64_t row = (int64_t)(j + 2) * we;
    const int x[4] = {(int)(row + i), (int)(row + i + 1), (int)(row + i + 2), (int)(row + i + 3)};
    const double g = c.gamma;
    const int64_t lo = (int64_t)(j + 1) * we, hi = (int64_t)(j + 3) * we;
    const UVT<double> uL = uvt_a(ldw(e, plane, x[1]), g), uR = uvt_a(ldw(e, plane, x[2]), g);
    const UVT<double> nA = avg4(uvt_a(ldw(e, plane, lo + i + 1), g), uvt_a(ldw(e, plane, lo + i + 2), g), uL, uR);
    const UVT<double> nB = avg4(uL, uR, uvt_a(ldw(e, plane, hi + i + 1), g), uvt_a(ldw(e, plane, hi + i + 2), g));
    double rl[4], rr[4];
    rbar_cell(B, rbar, n, i - 1, j, rl);
    rbar_cell(B, rbar, n, i, j, rr);
    const double Fb[4] = {rl[0] - rr[0], rl[1] - rr[1], rl[2] - rr[2], rl[3] - rr[3]};
    double sx = SI[2 * B.fi_off + f], sy = SI[2 * B.fi_off + nf + f];
    double dx = dI[2 * B.fi_off + f], dy = dI[2 * B.fi_off + nf + f];
    double vg = 0.0, gx = 0.0, gy = 0.0;
    MotionSnap m{1.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MV)
        vg = moving_geo(mo, B, n, xy, (int64_t)j * W + i, (int64_t)(j + 1) * W + i, sx, sy, dx, dy, m, gx, gy);
    face_rev<NT, MV, GEO>(e, plane, x, nA, nB, sx, sy, dx, dy, Fb, c,
             AF + B.afi_off + (int64_t)n * kAF * nf + f, nf, vg, &m, gx, gy,
             Mb ? Mb + B.afi_off / kAF * 2 + (int64_t)n * 2 * nf + f : nullptr, nf);
}

template <bool NT, bool MV, bool GEO>
__device__ __forceinline__ void adj_face_j(const BlockDesc *blks, int b, const double *ext, const double *SJ,
                             const double *dJ, const double *rbar, Consts c, double *AF, Motion mo,
                             const double *xy, double *Mb, int64_t tid_) {
    const BlockDesc &B = blks[b];
    const int64_t nf = (int64_t)B.ni * (B.nj + 1);
    const int64_t t = tid_;
    if (t >= nf * B.ns) return;
    const int n = (int)(t / nf);
    const int64_t f = t % nf;
    const int i = (int)(f % B.ni), j = (int)(f / B.ni);
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    const int col = i + 2;
    const int x[4] = {(int)((int64_t)j * we + col), (int)((int64_t)(j + 1) * we + col),
                      (int)((int64_t)(j + 2) * we + col), (int)((int64_t)(j + 3) * we + col)};
    const double g = c.gamma;
    const UVT<double> uL = uvt_a(ldw(e, plane, x[1]), g), uR = uvt_a(ldw(e, plane, x[2]), g);
    const int64_t r1 = (int64_t)(j + 1) * we, r2 = (int64_t)(j + 2) * we;
    const UVT<double> nA = avg4(uvt_a(ldw(e, plane, r1 + col - 1), g), uL,
                                uvt_a(ldw(e, plane, r2 + col - 1), g), uR);          // node (i, j)
    const UVT<double> nB = avg4(uL, uvt_a(ldw(e, plane, r1 + col + 1), g), uR,
                                uvt_a(ldw(e, plane, r2 + col + 1), g));              // node (i+1, j)
    double rl[4], rr[4];
    rbar_cell(B, rbar, n, i, j - 1, rl);
    rbar_cell(B, rbar, n, i, j, rr);
    const double Fb[4] = {rl[0] - rr[0], rl[1] - rr[1], rl[2] - rr[2], rl[3] - rr[3]};
    double sx = SJ[2 * B.fj_off + f], sy = SJ[2 * B.fj_off + nf + f];
    double dx = dJ[2 * B.fj_off + f], dy = dJ[2 * B.fj_off + nf + f];
    double vg = 0.0, gx = 0.0, gy = 0.0;
    MotionSnap m{1.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MV) {
        const int64_t kA = (int64_t)j * (B.ni + 1) + i;
        vg = moving_geo(mo, B, n, xy, kA, kA + 1, sx, sy, dx, dy, m, gx, gy);
    }
    face_rev<NT, MV, GEO>(e, plane, x, nB, nA, sx, sy, dx, dy, Fb, c,
             AF + B.afj_off + (int64_t)n * kAF * nf + f, nf, vg, &m, gx, gy,
             Mb ? Mb + B.afj_off / kAF * 2 + (int64_t)n * 2 * nf + f : nullptr, nf);
}

// one launch for both face families of block b: workgroup w takes i-face
// items [128 w, 128 w + 128) with its first half and the j-face items of the
// same range with its second (items snapshot-major, so both halves read the
// same rows of the same snapshot); xcd: XCD-aware workgroup order
// (launched with xcd_grid workgroups), else the launch order.  GEO: the S and
// d adjoints (records 22..25) are formed and stored, for the coordinate
// adjoints; without them that part of the reverse sweep is not compiled.
template <bool NT, bool MV, bool GEO>
__global__ void __launch_bounds__(kBS) k_adj_faces(const BlockDesc *blks, int b, const double *ext,
                                                   const double *SI, const double *dI,
                                                   const double *SJ, const double *dJ,
                                                   const double *rbar, Consts c, double *AFI,
                                                   double *AFJ, int64_t nI, int xcd, Motion mo,
                                                   const double *xy, double *MbI, double *MbJ) {
    const BlockDesc &B = blks[b];
    const int64_t nJ = (int64_t)B.ni * (B.nj + 1) * B.ns;
    constexpr int kHalf = kBS / 2;
    const int64_t W = ((nI > nJ ? nI : nJ) + kHalf - 1) / kHalf;
    const int64_t L = xcd ? xcd_group(W * kBS) : (int64_t)blockIdx.x;
    if (L < 0) return;
    const int64_t t = L * kHalf + (threadIdx.x % kHalf);
    if (threadIdx.x < kHalf) {
        if (t < nI) adj_face_i<NT, MV, GEO>(blks, b, ext, SI, dI, rbar, c, AFI, mo, xy, MbI, t);
    } else if (t < nJ) {
        adj_face_j<NT, MV, GEO>(blks, b, ext, SJ, dJ, rbar, c, AFJ, mo, xy, MbJ, t);
    }
}

// (u, v, T) adjoint of node (i, j) of one snapshot (ai, aj: that snapshot's
// i- and j-face records): the sum over the node's four faces in a fixed
// order.  Every load is issued (faces outside the block read face 0 and add
// zero), so that the four faces cost one memory round trip instead of four.
__device__ __forceinline__ UVT<double> node_adj(const BlockDesc &B, const double *ai, const double *aj,
                                                int64_t nfi, int64_t nfj, int i, int j) {
    const int W = B.ni + 1;
    const bool has[4] = {j < B.nj, j >= 1, i < B.ni, i >= 1};
    const double *src[4] = {
        ai + 16 * nfi + (has[0] ? (int64_t)j * W + i : 0),           // i-face (i, j): slot 0
        ai + 19 * nfi + (has[1] ? (int64_t)(j - 1) * W + i : 0),     // i-face (i, j-1): slot 1
        aj + 19 * nfj + (has[2] ? (int64_t)j * B.ni + i : 0),        // j-face (i, j): slot 1
        aj + 16 * nfj + (has[3] ? (int64_t)j * B.ni + i - 1 : 0)};   // j-face (i-1, j): slot 0
    double x[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 3; ++v) x[q][v] = src[q][v * (q < 2 ? nfi : nfj)];
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 3; ++v) s[v] += has[q] ? x[q][v] : 0.0;
    return UVT<double>{s[0], s[1], s[2]};
}

// node (u, v, T) adjoints: [ns][3][nj+1][ni+1]
// Also clears this block's node-coordinate adjoints (xyb, may be null),
// which the fold and coordinate kernels then accumulate.
__global__ void __launch_bounds__(kBS) k_adj_nodes(const BlockDesc *blks, int b, const double *AFI, const double *AFJ,
                            double *NB, double *xyb) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nn = (int64_t)W * (B.nj + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (xyb) {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t k = t; k < 2 * nn; k += stride) xyb[2 * B.node_off + k] = 0.0;
    }
    if (t >= nn * B.ns) return;
    const int n = (int)(t / nn);
    const int64_t k = t % nn;
    const int i = (int)(k % W), j = (int)(k / W);
    const int64_t nfi = (int64_t)W * B.nj, nfj = (int64_t)B.ni * (B.nj + 1);
    const UVT<double> s = node_adj(B, AFI + B.afi_off + (int64_t)n * kAF * nfi,
                                   AFJ + B.afj_off + (int64_t)n * kAF * nfj, nfi, nfj, i, j);
    double *o = NB + B.nodeq_off + (int64_t)n * 3 * nn + k;
    o[0] = s.u;
    o[nn] = s.v;
    o[2 * nn] = s.t;
}

// Primitive adjoint of ghost-extended cell t of a block (all snapshots
// flattened: [ns][4][nj+4][ni+4]); returns this cell's alpha0 adjoint term
// when it is a far-field ghost (ffc != 0) and alpha is asked for:
// d(u, v)/d alpha = (-v_inf, u_inf), a mirrored ghost flips both.
template <bool NI>
__device__ __forceinline__ double adj_cell(const BlockDesc &B, int64_t t, int we, int64_t plane,
                                           const double *ext, const double *AFI, const double *AFJ,
                                           const double *NB, const Consts &c, double *WB,
                                           const int8_t *ffc, const double *ffw, bool alpha) {
    const int n = (int)(t / plane);
    const int64_t r = t % plane;
    const int i = (int)(r % we) - 2, j = (int)(r / we) - 2;
    const int W = B.ni + 1;
    const int64_t nfi = (int64_t)W * B.nj, nfj = (int64_t)B.ni * (B.nj + 1);
    const int64_t nn = (int64_t)W * (B.nj + 1);
    const double *ai = AFI + B.afi_off + (int64_t)n * kAF * nfi;
    const double *aj = AFJ + B.afj_off + (int64_t)n * kAF * nfj;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    // line stencils: this cell is m2 of face +2, m1 of +1, p0 of +0, p1 of -1
    if (j >= 0 && j < B.nj) {
        for (int role = 0; role < 4; ++role) {
            const int f = i + 2 - role;
            if (f < 0 || f > B.ni) continue;
            const int64_t fi = (int64_t)j * W + f;
            for (int v = 0; v < 4; ++v) s[v] += ai[(role * 4 + v) * nfi + fi];
        }
    }
    if (i >= 0 && i < B.ni) {
        for (int role = 0; role < 4; ++role) {
            const int f = j + 2 - role;
            if (f < 0 || f > B.nj) continue;
            const int64_t fj = (int64_t)f * B.ni + i;
            for (int v = 0; v < 4; ++v) s[v] += aj[(role * 4 + v) * nfj + fj];
        }
    }
    // nodes (i, j), (i+1, j), (i, j+1), (i+1, j+1) average this cell; their
    // adjoints from the node kernel's array, or (NI) summed here from the
    // face records, the same sums in the same order
    UVT<double> nb{0.0, 0.0, 0.0};
    const double *nq = NB + B.nodeq_off + (int64_t)n * 3 * nn;
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const int a = i + di, bb = j + dj;
            if (a < 0 || a > B.ni || bb < 0 || bb > B.nj) continue;
            const int64_t k = (int64_t)bb * W + a;
            const UVT<double> na = NI ? node_adj(B, ai, aj, nfi, nfj, a, bb)
                                      : UVT<double>{nq[k], nq[nn + k], nq[2 * nn + k]};
            nb.u += 0.25 * na.u;
            nb.v += 0.25 * na.v;
            nb.t += 0.25 * na.t;
        }
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    W4<double> wb{s[0], s[1], s[2], s[3]};
    uvt_rev(ldw(e, plane, r), nb, c.gamma, wb);
    double *o = WB + B.ext_off + (int64_t)n * 4 * plane + r;
    o[0] = wb.r;
    o[plane] = wb.u;
    o[2 * plane] = wb.v;
    o[3 * plane] = wb.p;
    if (!alpha || ffc[r] == 0) return 0.0;
    const double *w = ffw + 4 * (B.snap_off + n);
    return (double)ffc[r] * (wb.u * -w[2] + wb.v * w[1]);
}

// primitive adjoints of every ghost-extended cell; with apart (may be null)
// also the alpha0 adjoint of the far-field ghosts as one partial per
// (logical) workgroup (fixed-order tree sum); xcd as for k_adj_faces.
// NI: the node adjoints are summed from the face records here instead of
// read from the node kernel's array (blocks whose records stay in the
// last-level cache; the node kernel's launch is then left out), and this
// kernel clears the block's node-coordinate adjoints (xyb, may be null).
template <bool NI>
__global__ void __launch_bounds__(kBS) k_adj_cells(const BlockDesc *blks, int b, const double *ext, const double *AFI,
                            const double *AFJ, const double *NB, Consts c, double *WB,
                            const int8_t *ffc, const double *ffw, double *apart, int xcd, double *xyb) {
    const BlockDesc &B = blks[b];
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    if (NI && xyb) {
        const int64_t nn2 = 2 * (int64_t)(B.ni + 1) * (B.nj + 1);
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn2; k += stride)
            xyb[2 * B.node_off + k] = 0.0;
    }
    const int64_t L = xcd ? xcd_group(plane * B.ns) : (int64_t)blockIdx.x;
    if (L < 0) return;                     // a whole padding workgroup
    const int64_t t = L * kBS + threadIdx.x;
    double acc = 0.0;
    if (t < plane * B.ns) acc = adj_cell<NI>(B, t, we, plane, ext, AFI, AFJ, NB, c, WB, ffc, ffw, apart != nullptr);
    if (apart) {
        __shared__ double red[kBS];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kBS / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) apart[L] = red[0];
    }
}

// The cell's state and own ghost-extended adjoint of snapshot n (t = cell
// of block B).
struct FoldIn {
    double q[4], w[4];
};
__device__ __forceinline__ FoldIn fold_load(const BlockDesc &B, int64_t t, int n, const double *q,
                                            const double *WB) {
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int i = (int)(t % B.ni), j = (int)(t / B.ni);
    const int we = B.ni + 4;
    const int64_t eplane = (int64_t)we * (B.nj + 4);
    const int64_t own = (int64_t)(j + 2) * we + i + 2;
    const double *qc = q + B.q_off + (int64_t)n * 4 * plane + t;
    const double *wbn = WB + B.ext_off + (int64_t)n * 4 * eplane + own;
    FoldIn r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        r.q[v] = qc[v * plane];
        r.w[v] = wbn[v * eplane];
    }
    return r;
}

// Snapshot n of cell t: the ghost copies [k0, k1) of the fold list added to
// the own adjoint, the primitive-to-conserved transpose, plus V (D^T rbar)
// (hw); stores q-bar and returns the cell-area term Q . hw.
__device__ __forceinline__ double fold_finish(const BlockDesc *blks, const BlockDesc &B, int64_t t, int n,
                                              const FoldIn &in, const double *WB, int k0, int k1,
                                              const int *fb, const int *fp, const int *fm, double vol,
                                              const Consts &c, const double hw[4], double *qbar) {
    const int64_t plane = (int64_t)B.ni * B.nj;
    const double gm1 = c.gamma - 1.0;
    const double *qn = in.q;
    double wbv[4] = {in.w[0], in.w[1], in.w[2], in.w[3]};
    for (int k = k0; k < k1; ++k) {
        const BlockDesc &S = blks[fb[k]];
        const int64_t sp = (int64_t)(S.ni + 4) * (S.nj + 4);
        const double *ws = WB + S.ext_off + (int64_t)n * 4 * sp + fp[k];
        const double sg = fm[k] ? -1.0 : 1.0;
        wbv[0] += ws[0];
        wbv[1] += sg * ws[sp];
        wbv[2] += sg * ws[2 * sp];
        wbv[3] += ws[3 * sp];
    }
    const double irq = adj_rcp(qn[0]);
    const W4<double> w{qn[0], qn[1] * irq, qn[2] * irq,
                       gm1 * (qn[3] - 0.5 * qn[0] * (qn[1] * irq * qn[1] * irq + qn[2] * irq * qn[2] * irq))};
    double qb[4];
    prim_rev(w, W4<double>{wbv[0], wbv[1], wbv[2], wbv[3]}, gm1, qb);
    double *o = qbar + B.q_off + (int64_t)n * 4 * plane + t;
    double vb = 0.0;
    for (int v = 0; v < 4; ++v) {
        o[v * plane] = qb[v] + vol * hw[v];
        vb += qn[v] * hw[v];
    }
    return vb;
}

__device__ __forceinline__ double fold_one(const BlockDesc *blks, const BlockDesc &B, int64_t t, int n,
                                           const double *q, const double *WB, const int *fptr,
                                           const int *fb, const int *fp, const int *fm, double vol,
                                           const Consts &c, const double hw[4], double *qbar) {
    const int64_t gc = B.cell_off + t;
    const FoldIn in = fold_load(B, t, n, q, WB);
    return fold_finish(blks, B, t, n, in, WB, fptr[gc], fptr[gc + 1], fb, fp, fm, vol, c, hw, qbar);
}

// interior cells: own adjoint + ghost copies -> conserved adjoint + HB
// source D^T rbar (d/dQ_n of sum_m rbar_m V (D Q)_m = V (D^T rbar)_n); with
// VB also the adjoint of the cell area from the HB source, rbar . (D Q),
// stored per cell for the coordinate node gather (rbar == nullptr: no HB
// source).
// PER_SNAP: one thread per cell and snapshot (small blocks, which would
// otherwise leave CUs idle), each writing its snapshot's share of the
// cell-area adjoint to VB[n * vbs + cell]; a workgroup takes all snapshots
// of C = kBS / N_s consecutive cells (thread n C + c), whose rbar it stages
// in LDS once for the D^T rbar sums.  Else one thread per cell looping over
// the snapshots with the cell's rbar in registers, writing VB[cell].
__device__ __forceinline__ void adj_xy_i(const BlockDesc *blks, int b, const double *AF, const double *Mb,
                           const double *xy, const double *C, double *xyb, double *G, int64_t n_fi,
                           int64_t tid_);
__device__ __forceinline__ void adj_xy_j(const BlockDesc *blks, int b, const double *AF, const double *Mb,
                           const double *xy, const double *C, double *xyb, double *G, int64_t n_fj,
                           int64_t tid_);

// The per-face step of the coordinate adjoints (adj_xy_i/j) of one block,
// run by the workgroups of a fold launch past its fold workgroups: the two
// are independent (the face step reads the face records and adds into the
// node adjoints that the node kernel has cleared), so one launch covers both
// and the short face step fills the fold's tail.
struct XyStep {
    const double *AFI, *AFJ, *MbI, *MbJ, *xy, *C;
    double *xyb, *G;
    int64_t n_fi, n_fj, nI, n;     // n = i-faces + j-faces of the block; 0: no face step
    unsigned first;                // first workgroup of the face step
};

template <bool PER_SNAP>
__global__ void __launch_bounds__(kBS) k_adj_fold(const BlockDesc *blks, int b, const double *q,
                                                  const double *rbar, const double *WB,
                                                  const int *fptr, const int *fb, const int *fp,
                                                  const int *fm, const double *V, const double *D,
                                                  Consts c, double *qbar, const double *apart,
                                                  int64_t napart, double *flowbar, double *VB,
                                                  int64_t vbs, XyStep xs) {
    if (xs.n && blockIdx.x >= xs.first) {
        const int64_t t = (int64_t)(blockIdx.x - xs.first) * kBS + threadIdx.x;
        if (t < xs.nI) adj_xy_i(blks, b, xs.AFI, xs.MbI, xs.xy, xs.C, xs.xyb, xs.G, xs.n_fi, t);
        else if (t < xs.n)
            adj_xy_j(blks, b, xs.AFJ, xs.MbJ, xs.xy, xs.C, xs.xyb, xs.G + 6 * xs.n_fi, xs.n_fj, t - xs.nI);
        return;
    }
    // workgroup 0 (of the first block's launch) first sums the alpha0
    // partials of the cell-adjoint kernels, in a fixed order
    if (flowbar && blockIdx.x == 0) {
        __shared__ double red[kBS];
        double acc = 0.0;
        for (int64_t k = threadIdx.x; k < napart; k += kBS) acc += apart[k];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s2 = kBS / 2; s2 > 0; s2 >>= 1) {
            if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
            __syncthreads();
        }
        if (threadIdx.x == 0) *flowbar = red[0];
    }
    const BlockDesc &B = blks[b];
    // the block's D (N_s x N_s of the kNsPad x kNsPad table) in LDS: every
    // thread reads all of it
    __shared__ double dm[kMaxNs * kNsPad];
    for (int k = threadIdx.x; k < kMaxNs * kNsPad; k += blockDim.x) dm[k] = D[B.d_off + k];
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int ns = B.ns;
    if constexpr (PER_SNAP) {
        __shared__ double rbs[4 * kBS];            // rbs[(m 4 + v) C + c]
        const int C = kBS / ns, tid = (int)threadIdx.x;
        const int cg = tid % C, n = tid / C;
        const int64_t t = (int64_t)blockIdx.x * C + cg;
        const bool live = n < ns && t < plane;
        if (live)
            for (int v = 0; v < 4; ++v)
                rbs[(n * 4 + v) * C + cg] = rbar ? rbar[B.q_off + ((int64_t)n * 4 + v) * plane + t] : 0.0;
        __syncthreads();
        if (!live) return;
        double hw[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = 0; m < ns; ++m) {
            const double d = dm[m * kNsPad + n];
#pragma unroll
            for (int v = 0; v < 4; ++v) hw[v] += d * rbs[(m * 4 + v) * C + cg];
        }
        const int64_t gc = B.cell_off + t;
        const double vb = fold_one(blks, B, t, n, q, WB, fptr, fb, fp, fm, V[gc], c, hw, qbar);
        if (VB) VB[(int64_t)n * vbs + gc] = rbar ? vb : 0.0;
    } else {
        __syncthreads();
        const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (t >= plane) return;
        const int64_t gc = B.cell_off + t;
        const double vol = V[gc];
        // rbar of this cell, all snapshots, in registers (static indices only)
        double rb[kMaxNs][4];
#pragma unroll
        for (int m = 0; m < kMaxNs; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                rb[m][v] = (rbar && m < ns) ? rbar[B.q_off + ((int64_t)m * 4 + v) * plane + t] : 0.0;
        double vb = 0.0;
        // the next snapshot's loads are issued before this snapshot's
        // arithmetic and stores (one memory round trip per snapshot is
        // otherwise exposed)
        const int k0 = fptr[gc], k1 = fptr[gc + 1];
        FoldIn nx = fold_load(B, t, 0, q, WB);
        for (int n = 0; n < ns; ++n) {
            const FoldIn cur = nx;
            if (n + 1 < ns) nx = fold_load(B, t, n + 1, q, WB);
            double hw[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int m = 0; m < kMaxNs; ++m) {
                if (m < ns) {
                    const double d = dm[m * kNsPad + n];
#pragma unroll
                    for (int v = 0; v < 4; ++v) hw[v] += d * rb[m][v];
                }
            }
            vb += fold_finish(blks, B, t, n, cur, WB, k0, k1, fb, fp, fm, vol, c, hw, qbar);
        }
        // adjoint of the cell area (its node derivatives are taken by the
        // coordinate node gather)
        if (VB) VB[gc] = rbar ? vb : 0.0;
    }
}

// alpha0: far-field ghost adjoints . d w_inf / d alpha0; one thread per
// (far-field ghost, snapshot) of block b, one partial per workgroup (summed
// in a fixed order afterwards)
__global__ void __launch_bounds__(kBS) k_adj_alpha(const BlockDesc *blks, int b, const double *WB,
                                                   const int *ffptr, const int *ffp, const int *ffm,
                                                   const double *ffw, double *part) {
    const BlockDesc &B = blks[b];
    const int k0 = ffptr[b], cnt = ffptr[b + 1] - k0;
    const int we = B.ni + 4;
    const int64_t eplane = (int64_t)we * (B.nj + 4);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (cnt > 0 && t < (int64_t)cnt * B.ns) {
        const int n = (int)(t / cnt), k = k0 + (int)(t % cnt);
        const double *w = ffw + 4 * (B.snap_off + n);
        // d(u, v)/d alpha = (-v_inf, u_inf); a mirrored far-field ghost flips both
        const double du = -w[2], dv = w[1];
        const double *wbn = WB + B.ext_off + (int64_t)n * 4 * eplane;
        const double sg = ffm[k] ? -1.0 : 1.0;
        acc = sg * (wbn[eplane + ffp[k]] * du + wbn[2 * eplane + ffp[k]] * dv);
    }
    __shared__ double red[kBS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *part, int n, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += part[k];
        *out = s;
    }
}

__global__ void k_zero(double *p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

// ---- node coordinates ------------------------------------------------------
__device__ inline void xadd(double *xb, int64_t idx, double v) { unsafeAtomicAdd(xb + idx, v); }

// add a centre adjoint (cx, cy) of cell (i, j) of block b to its four nodes
__device__ inline void centre_to_nodes(const BlockDesc *blks, int b, int i, int j, double cx,
                                       double cy, double *xyb) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nn = (int64_t)W * (B.nj + 1);
    double *xb = xyb + 2 * B.node_off;
    double *yb = xb + nn;
    const int64_t k0 = (int64_t)j * W + i;
    const int64_t ks[4] = {k0, k0 + 1, k0 + W, k0 + W + 1};
    for (int k = 0; k < 4; ++k) {
        xadd(xb, ks[k], 0.25 * cx);
        xadd(yb, ks[k], 0.25 * cy);
    }
}

// adjoint of P' = reflect(P, A, B) -> P, A, B
__device__ inline void reflect_rev(double px, double py, double ax, double ay, double bx, double by,
                                   double rbx, double rby, double &pbx, double &pby, double &abx,
                                   double &aby, double &bbx, double &bby) {
    const double ex = bx - ax, ey = by - ay;
    const double num = (px - ax) * ex + (py - ay) * ey;
    const double den = ex * ex + ey * ey;
    const double t = num / den;
    abx += 2.0 * rbx;
    aby += 2.0 * rby;
    pbx -= rbx;
    pby -= rby;
    double ebx = 2.0 * t * rbx, eby = 2.0 * t * rby;
    const double tb = 2.0 * (rbx * ex + rby * ey);
    const double numb = tb / den, denb = -tb * num / (den * den);
    pbx += numb * ex;
    pby += numb * ey;
    abx -= numb * ex;
    aby -= numb * ey;
    ebx += numb * (px - ax) + 2.0 * denb * ex;
    eby += numb * (py - ay) + 2.0 * denb * ey;
    bbx += ebx;
    bby += eby;
    abx -= ebx;
    aby -= eby;
}

// Ghost-centre adjoint of a boundary face: (gx, gy) is the adjoint of the
// ghost cell's centre; side = block side; (ii, jj) = the interior cell next
// to the face; A, B = face end nodes (indices into the block's nodes).
__device__ inline void ghost_centre_rev(const BlockDesc *blks, int b, int side, int ii, int jj,
                                        int kA, int kB, double gx, double gy, const double *xy,
                                        const double *C, double *xyb) {
    const BlockDesc &B = blks[b];
    const int kind = B.bc[side];
    const bool wake = side == 2 && kind == HB_BC_WAKECUT && (ii < B.wake || ii >= B.ni - B.wake);
    if (kind == HB_BC_PERIODIC) {
        const int pi = side == 0 ? B.ni - 1 : side == 1 ? 0 : ii;
        const int pj = side == 2 ? B.nj - 1 : side == 3 ? 0 : jj;
        centre_to_nodes(blks, b, pi, pj, gx, gy, xyb);
    } else if (wake) {
        centre_to_nodes(blks, b, B.ni - 1 - ii, 0, gx, gy, xyb);
    } else if (glued_at(B, B.segs, side, side < 2 ? jj : ii)) {
        int a, pi, pj;
        cut_cell(blks, B.segs, b, side, 0, side < 2 ? jj : ii, &a, &pi, &pj);
        centre_to_nodes(blks, a, pi, pj, gx, gy, xyb);
    } else {   // wall or far field: mirror of the interior centre across the face
        const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
        const double *x = xy + 2 * B.node_off, *y = x + nn;
        const int64_t nc = (int64_t)B.ni * B.nj;
        const int64_t ci = B.cell_off + (int64_t)jj * B.ni + ii;
        const double px = C[2 * B.cell_off + (ci - B.cell_off)];
        const double py = C[2 * B.cell_off + nc + (ci - B.cell_off)];
        double pbx = 0, pby = 0, abx = 0, aby = 0, bbx = 0, bby = 0;
        reflect_rev(px, py, x[kA], y[kA], x[kB], y[kB], gx, gy, pbx, pby, abx, aby, bbx, bby);
        centre_to_nodes(blks, b, ii, jj, pbx, pby, xyb);
        double *xb = xyb + 2 * B.node_off;
        double *yb = xb + nn;
        xadd(xb, kA, abx);
        xadd(yb, kA, aby);
        xadd(xb, kB, bbx);
        xadd(yb, kB, bby);
    }
}

// Coordinate adjoints, in two steps.  Per face: the adjoints of S and d
// summed over the snapshots are stored (G), and the ghost side of a face on
// a block side goes through ghost_centre_rev (atomic adds, possibly into a
// neighbour block).  Per node: the face-length parts of the (up to) four
// faces at the node, the centre parts of the (up to) four cells around it
// (a cell centre is the mean of its nodes; its adjoint is the sum over its
// faces of +d for the faces where it is R and -d where it is L) and the cell
// areas' adjoints (VB, from the HB source) are gathered and added, without
// atomics.
// The S and d adjoints of one face (and, with Mb, its midpoint adjoints)
// summed over the ns snapshots in snapshot order.  Every snapshot's loads
// are issued before the first sum: a loop that adds as it loads waits for
// one memory round trip per snapshot.
__device__ __forceinline__ void sum_face_snapshots(const double *a, const double *mb, int64_t nf, int ns,
                                                   double &sxb, double &syb, double &dxb, double &dyb,
                                                   double &mxb, double &myb) {
    double v[kMaxNs][4];
#pragma unroll
    for (int n = 0; n < kMaxNs; ++n) {
        if (n < ns) {
            const double *an = a + (int64_t)n * kAF * nf;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[n][c] = an[(22 + c) * nf];
        }
    }
#pragma unroll
    for (int n = 0; n < kMaxNs; ++n) {
        if (n < ns) {
            sxb += v[n][0];
            syb += v[n][1];
            dxb += v[n][2];
            dyb += v[n][3];
        }
    }
    if (mb) {
        for (int n = 0; n < ns; ++n) {
            mxb += mb[(int64_t)n * 2 * nf];
            myb += mb[(int64_t)n * 2 * nf + nf];
        }
    }
}

// i-faces: S_I = (yB - yA, xA - xB), A = node (i, j), B = node (i, j+1);
// d = centre(R) - centre(L)
__device__ __forceinline__ void adj_xy_i(const BlockDesc *blks, int b, const double *AF, const double *Mb,
                           const double *xy, const double *C, double *xyb, double *G, int64_t n_fi,
                           int64_t tid_) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nf = (int64_t)W * B.nj;
    const int64_t f = tid_;
    if (f >= nf) return;
    const int i = (int)(f % W), j = (int)(f / W);
    double sxb = 0, syb = 0, dxb = 0, dyb = 0, mxb = 0, myb = 0;
    sum_face_snapshots(AF + B.afi_off + f, Mb ? Mb + B.afi_off / kAF * 2 + f : nullptr, nf, B.ns,
                       sxb, syb, dxb, dyb, mxb, myb);
    double *g = G + B.fi_off + f;
    g[0] = sxb;
    g[n_fi] = syb;
    g[2 * n_fi] = dxb;
    g[3 * n_fi] = dyb;
    g[4 * n_fi] = mxb;
    g[5 * n_fi] = myb;
    const int64_t kA = (int64_t)j * W + i, kB = kA + W;
    if (i == B.ni) ghost_centre_rev(blks, b, 1, B.ni - 1, j, (int)kA, (int)kB, dxb, dyb, xy, C, xyb);
    if (i == 0) ghost_centre_rev(blks, b, 0, 0, j, (int)kA, (int)kB, -dxb, -dyb, xy, C, xyb);
}

// j-faces: S_J = (yA - yB, xB - xA), A = node (i, j), B = node (i+1, j)
__device__ __forceinline__ void adj_xy_j(const BlockDesc *blks, int b, const double *AF, const double *Mb,
                           const double *xy, const double *C, double *xyb, double *G, int64_t n_fj,
                           int64_t tid_) {
    const BlockDesc &B = blks[b];
    const int W = B.ni + 1;
    const int64_t nf = (int64_t)B.ni * (B.nj + 1);
    const int64_t f = tid_;
    if (f >= nf) return;
    const int i = (int)(f % B.ni), j = (int)(f / B.ni);
    double sxb = 0, syb = 0, dxb = 0, dyb = 0, mxb = 0, myb = 0;
    sum_face_snapshots(AF + B.afj_off + f, Mb ? Mb + B.afj_off / kAF * 2 + f : nullptr, nf, B.ns,
                       sxb, syb, dxb, dyb, mxb, myb);
    double *g = G + B.fj_off + f;
    g[0] = sxb;
    g[n_fj] = syb;
    g[2 * n_fj] = dxb;
    g[3 * n_fj] = dyb;
    g[4 * n_fj] = mxb;
    g[5 * n_fj] = myb;
    const int64_t kA = (int64_t)j * W + i, kB = kA + 1;
    if (j == B.nj) ghost_centre_rev(blks, b, 3, i, B.nj - 1, (int)kA, (int)kB, dxb, dyb, xy, C, xyb);
    if (j == 0) ghost_centre_rev(blks, b, 2, i, 0, (int)kA, (int)kB, -dxb, -dyb, xy, C, xyb);
}

// per-face step for both face families of block b in one launch
// (per face: G holds the S, d and, on a moving grid, midpoint adjoints
// summed over the snapshots, [6][n_fi] then [6][n_fj])
__global__ void __launch_bounds__(kBS) k_adj_xy(const BlockDesc *blks, int b, const double *AFI,
                                                const double *AFJ, const double *MbI,
                                                const double *MbJ, const double *xy, const double *C,
                                                double *xyb, double *G, int64_t n_fi, int64_t n_fj,
                                                int64_t nI) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nI) adj_xy_i(blks, b, AFI, MbI, xy, C, xyb, G, n_fi, t);
    else adj_xy_j(blks, b, AFJ, MbJ, xy, C, xyb, G + 6 * n_fi, n_fj, t - nI);
}

// per-node step: four lanes per node of block b.  Lane c of a node takes
// the node's face c (i-face above, i-face below, j-face right, j-face left)
// and the cell at its corner c (cells (i, j), (i-1, j), (i-1, j-1),
// (i, j-1), where the node is that cell's corner 1, 2, 3, 4); the four
// partial sums are combined by two lane exchanges, a fixed order.
__global__ void __launch_bounds__(kBS) k_adj_xy_nodes(const BlockDesc *blks, int b, const double *G,
                                                      int64_t n_fi, int64_t n_fj, const double *VB,
                                                      int nvb, int64_t vbs, const double *xy,
                                                      int mid, double *xyb) {
    const BlockDesc &B = blks[b];
    const int ni = B.ni, nj = B.nj, W = ni + 1;
    const int64_t nn = (int64_t)W * (nj + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = t >> 2;
    const int c = (int)(t & 3);
    const bool on = k < nn;
    const int i = on ? (int)(k % W) : 0, j = on ? (int)(k / W) : 0;
    // the sign of this lane's face and corner terms: - for lanes 0 and 3
    const double sg = (c == 0 || c == 3) ? -1.0 : 1.0;
    double ax = 0.0, ay = 0.0;
    // face length (and, on a moving grid, half of the face's midpoint
    // adjoint): S_I = (yB - yA, xA - xB) with this node as A of i-face
    // (i, j) and B of i-face (i, j-1); S_J = (yA - yB, xB - xA) with it as A
    // of j-face (i, j) and B of j-face (i-1, j)
    {
        const bool fI = c < 2;
        const int fi = c == 3 ? i - 1 : i, fj = c == 1 ? j - 1 : j;
        const bool fin = on && (c == 0 ? j < nj : c == 1 ? j > 0 : c == 2 ? i < ni : i > 0);
        if (fin) {
            const int64_t st = fI ? n_fi : n_fj;
            const double *gf = fI ? G + B.fi_off + (int64_t)fj * W + fi
                                  : G + 6 * n_fi + B.fj_off + (int64_t)fj * ni + fi;
            ay += sg * gf[0];
            ax -= sg * gf[st];
            if (mid) {
                ax += 0.5 * gf[4 * st];
                ay += 0.5 * gf[5 * st];
            }
        }
    }
    // cell at corner c: its centre (the mean of its nodes) and, with VB, its
    // area V = ((x3 - x1)(y4 - y2) - (y3 - y1)(x4 - x2)) / 2 over its nodes
    // 1 = (ci, cj), 2 = (ci+1, cj), 3 = (ci+1, cj+1), 4 = (ci, cj+1)
    {
        const int ci = (c == 1 || c == 2) ? i - 1 : i, cj = c >= 2 ? j - 1 : j;
        const bool cin = on && ci >= 0 && ci < ni && cj >= 0 && cj < nj;
        if (cin) {
            const double *gi = G + B.fi_off, *gj = G + 6 * n_fi + B.fj_off;
            const int64_t fa = (int64_t)cj * W + ci, fb = (int64_t)cj * ni + ci;
            ax += 0.25 * (gi[2 * n_fi + fa] - gi[2 * n_fi + fa + 1] + gj[2 * n_fj + fb] - gj[2 * n_fj + fb + ni]);
            ay += 0.25 * (gi[3 * n_fi + fa] - gi[3 * n_fi + fa + 1] + gj[3 * n_fj + fb] - gj[3 * n_fj + fb + ni]);
            if (VB) {
                const double *vb = VB + B.cell_off + (int64_t)cj * ni + ci;
                double vs[kMaxNs];
#pragma unroll
                for (int m = 0; m < kMaxNs; ++m)
                    if (m < nvb) vs[m] = vb[(int64_t)m * vbs];
                double vsum = 0.0;
#pragma unroll
                for (int m = 0; m < kMaxNs; ++m)
                    if (m < nvb) vsum += vs[m];
                const double h = 0.5 * vsum;
                // the two other corners this node's term uses: 4 and 2 for
                // corners 1 and 3, 3 and 1 for corners 2 and 4
                const double *x = xy + 2 * B.node_off, *y = x + nn;
                const int64_t k1 = (int64_t)cj * W + ci;
                const int64_t kp = (c & 1) ? k1 + W + 1 : k1 + W, km = (c & 1) ? k1 : k1 + 1;
                ax += sg * h * (y[kp] - y[km]);
                ay -= sg * h * (x[kp] - x[km]);
            }
        }
    }
    ax += __shfl_xor(ax, 1);
    ay += __shfl_xor(ay, 1);
    ax += __shfl_xor(ax, 2);
    ay += __shfl_xor(ay, 2);
    if (on && c == 0) {
        double *xb = xyb + 2 * B.node_off;
        xb[k] += ax;
        xb[nn + k] += ay;
    }
}

// Moving no-slip wall images u_g = 2 u_wall - u, u_wall the grid velocity at
// the body-frame midpoint of a wall face: the midpoint's adjoint from the
// ghost's velocity adjoint (WB), half to each node of the face.  One thread
// per ghost of the j-side ghost rows and snapshot; atomic adds (a wall face
// serves both ghost layers, and corner ghosts of neighbouring columns).
__global__ void __launch_bounds__(kBS) k_adj_wall_motion(const BlockDesc *blks, int b, const double *WB,
                                                         Motion mo, double *xyb) {
    const BlockDesc &B = blks[b];
    const int we = B.ni + 4;
    const int64_t eplane = (int64_t)we * (B.nj + 4);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)4 * we * B.ns) return;
    const int n = (int)(t / (4 * we)), r = (int)((t / we) % 4), ie = (int)(t % we);
    const int j = r < 2 ? r - 2 : B.nj + r - 2, i = ie - 2;
    int s;
    int64_t k;
    if (!wall_image_face(blks, b, i, j, &s, &k)) return;
    const double *wb = WB + B.ext_off + (int64_t)n * 4 * eplane + (int64_t)(j + 2) * we + ie;
    const MotionSnap m = motion_snap(mo, B, n);
    double xb, yb;
    grid_velocity_rev(m, 2.0 * wb[eplane], 2.0 * wb[2 * eplane], xb, yb);
    const BlockDesc &S = blks[s];
    const int64_t nn = (int64_t)(S.ni + 1) * (S.nj + 1);
    double *xs = xyb + 2 * S.node_off, *ys = xs + nn;
    atomicAdd(xs + k, 0.5 * xb);
    atomicAdd(xs + k + 1, 0.5 * xb);
    atomicAdd(ys + k, 0.5 * yb);
    atomicAdd(ys + k + 1, 0.5 * yb);
}

// ---- force coefficients ------------------------------------------------------

struct ForceAdj {
    const double *cfbar;      // [body][n][3] = (cl, cd, cm) adjoints
    const int *body_off;      // first entry of each body in cf
    double ca, sa;            // cos / sin of alpha0
    double qinf_l, qinf_l2;   // q_inf L, q_inf L^2
    double xm, ym;            // moment reference point
};

// One thread per jmin face and snapshot: the per-face record of the wall
// loads (zero for faces that are not wall), and the moment-arm adjoints.
// Face (i, 0): line cells (i, -2), (i, -1) [ghost, L], (i, 0) [wall cell, R],
// (i, 1); slot 0 = node (i+1, 0), slot 1 = node (i, 0), as in adj_face_j.
__global__ void __launch_bounds__(kBS) k_adj_force_face(const BlockDesc *blks, int b, const double *ext, const double *xy,
                                 const double *SJ, const double *dJ, ForceAdj fa, Consts c,
                                 double *AF, double *xyb, Motion mo) {
    const BlockDesc &B = blks[b];
    const int64_t nf = (int64_t)B.ni * (B.nj + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B.ni * B.ns) return;
    const int n = (int)(t / B.ni), i = (int)(t % B.ni);
    if (!jmin_wall(B, i)) return;
    const int we = B.ni + 4;
    const int64_t plane = (int64_t)we * (B.nj + 4);
    const double *e = ext + B.ext_off + (int64_t)n * 4 * plane;
    const int col = i + 2;
    const int64_t r1 = we, r2 = 2 * (int64_t)we;          // rows of cells j = -1 and j = 0
    const double g = c.gamma;
    const W4<double> wL = ldw(e, plane, r1 + col), wR = ldw(e, plane, r2 + col);
    const UVT<double> uL = uvt(wL, g), uR = uvt(wR, g);
    const UVT<double> nA = avg4(uvt(ldw(e, plane, r1 + col - 1), g), uL,
                                uvt(ldw(e, plane, r2 + col - 1), g), uR);          // node (i, 0)
    const UVT<double> nB = avg4(uL, uvt(ldw(e, plane, r1 + col + 1), g), uR,
                                uvt(ldw(e, plane, r2 + col + 1), g));              // node (i+1, 0)
    double sx = SJ[2 * B.fj_off + i], sy = SJ[2 * B.fj_off + nf + i];
    double dx = dJ[2 * B.fj_off + i], dy = dJ[2 * B.fj_off + nf + i];
    MotionSnap ms{1.0, 0.0, 0.0, 0.0, 0.0};
    if (mo.tab) {   // the snapshot's grid: body-frame vectors rotated by theta_n
        ms = motion_snap(mo, B, n);
        rot2(ms, sx, sy);
        rot2(ms, dx, dy);
    }
    double fv[3];
    viscous_flux(uL, uR, nB, nA, sx, sy, dx, dy, c.mu, c.kappa, fv);
    const double dp = wR.p - c.pinf;
    const double fx = -dp * sx + fv[0], fy = -dp * sy + fv[1];
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
    const double *x = xy + 2 * B.node_off, *y = x + nn;
    double mx = 0.5 * (x[i] + x[i + 1]) - fa.xm, my = 0.5 * (y[i] + y[i + 1]) - fa.ym;
    if (mo.tab) rot2(ms, mx, my);
    // coefficient adjoints -> (Fx, Fy, Mz) adjoints of this body and snapshot
    const double *cb = fa.cfbar + fa.body_off[B.body] + 3 * n;
    const double Fxb = (-cb[0] * fa.sa + cb[1] * fa.ca) / fa.qinf_l;
    const double Fyb = (cb[0] * fa.ca + cb[1] * fa.sa) / fa.qinf_l;
    const double Mzb = -cb[2] / fa.qinf_l2;
    // Mz = mx fy - my fx
    const double fxb = Fxb - my * Mzb, fyb = Fyb + mx * Mzb;
    if (xyb) {
        double mxb = 0.5 * Mzb * fy, myb = -0.5 * Mzb * fx;
        if (mo.tab) rot2_rev(ms, mxb, myb);   // the arm rotates with the body
        double *xb = xyb + 2 * B.node_off, *yb = xb + nn;
        xadd(xb, i, mxb);
        xadd(xb, i + 1, mxb);
        xadd(yb, i, myb);
        xadd(yb, i + 1, myb);
    }
    const double fvb[3] = {fxb, fyb, 0.0};
    UVT<double> uLb{0, 0, 0}, uRb{0, 0, 0}, Pb{0, 0, 0}, Qb{0, 0, 0};
    double sxb = -dp * fxb, syb = -dp * fyb, dxb = 0.0, dyb = 0.0;
    viscous_flux_rev(uL, uR, nB, nA, sx, sy, dx, dy, c.mu, c.kappa, fvb, uLb, uRb, Pb, Qb, sxb, syb,
                     dxb, dyb);
    if (mo.tab) {   // S and d adjoints back to the body frame
        rot2_rev(ms, sxb, syb);
        rot2_rev(ms, dxb, dyb);
    }
    W4<double> w1{0, 0, 0, 0}, w2{0, 0, 0, -(fxb * sx + fyb * sy)};
    uvt_rev(wL, uLb, g, w1);
    uvt_rev(wR, uRb, g, w2);
    double *o = AF + B.afj_off + (int64_t)n * kAF * nf + i;    // face (i, 0)
    const double cm1[4] = {w1.r, w1.u, w1.v, w1.p}, cp0[4] = {w2.r, w2.u, w2.v, w2.p};
    for (int v = 0; v < 4; ++v) {
        o[(4 + v) * nf] = cm1[v];
        o[(8 + v) * nf] = cp0[v];
    }
    o[16 * nf] = Pb.u;
    o[17 * nf] = Pb.v;
    o[18 * nf] = Pb.t;
    o[19 * nf] = Qb.u;
    o[20 * nf] = Qb.v;
    o[21 * nf] = Qb.t;
    o[22 * nf] = sxb;
    o[23 * nf] = syb;
    o[24 * nf] = dxb;
    o[25 * nf] = dyb;
}

// alpha0 through the wind axes: sum over entries of cdbar * cl - clbar * cd
__global__ void __launch_bounds__(kBS) k_adj_force_axes(const double *cf, const double *cfbar, int n, double *out) {
    __shared__ double red[kBS];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += kBS) acc += cfbar[3 * k + 1] * cf[3 * k] - cfbar[3 * k] * cf[3 * k + 1];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ---- adjoint pseudo-time iteration --------------------------------------------
// dtau / V per cell and snapshot of the (fixed) state q: the forward
// iteration's local step, laid out like one variable of the state.
__global__ void __launch_bounds__(kBS) k_adj_dtv(const BlockDesc *blks, int b, const double *q, const double *SI,
                          const double *SJ, const double *V, Consts c, double *dtv, Motion mo,
                          const double *C) {
    const BlockDesc &B = blks[b];
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= plane) return;
    const int i = (int)(t % B.ni), j = (int)(t / B.ni);
    const int W = B.ni + 1;
    const int64_t nfi = (int64_t)W * B.nj, nfj = (int64_t)B.ni * (B.nj + 1);
    const int64_t fi0 = (int64_t)j * W + i;
    const double vol = V[B.cell_off + t];
    const double sxi = 0.5 * (SI[2 * B.fi_off + fi0] + SI[2 * B.fi_off + fi0 + 1]);
    const double syi = 0.5 * (SI[2 * B.fi_off + nfi + fi0] + SI[2 * B.fi_off + nfi + fi0 + 1]);
    const double sxj = 0.5 * (SJ[2 * B.fj_off + t] + SJ[2 * B.fj_off + t + B.ni]);
    const double syj = 0.5 * (SJ[2 * B.fj_off + nfj + t] + SJ[2 * B.fj_off + nfj + t + B.ni]);
    for (int n = 0; n < B.ns; ++n) {
        const double *qc = q + B.q_off + (int64_t)n * 4 * plane + t;
        W4<double> w = prim_from_cons<double>(qc[0], qc[plane], qc[2 * plane], qc[3 * plane],
                                              c.gamma - 1.0);
        double ax = sxi, ay = syi, bx = sxj, by = syj;
        if (mo.tab) {   // snapshot's normals, velocity relative to the grid at the centre
            const MotionSnap m = motion_snap(mo, B, n);
            rot2(m, ax, ay);
            rot2(m, bx, by);
            double gx, gy;
            grid_velocity(m, mo, C[2 * B.cell_off + t], C[2 * B.cell_off + plane + t], gx, gy);
            w.u -= gx;
            w.v -= gy;
        }
        const double dt = local_dt<double>(w, ax, ay, bx, by, vol, c.gamma, c.mu / c.prandtl,
                                           c.cfl, B.omega_nh);
        dtv[B.q_off / 4 + (int64_t)n * plane + t] = dt / vol;
    }
}

// lam = lam0 - alpha (dtau/V) (J^T lam_in + gq); at the first stage the
// workgroup's partial sum of ((J^T lam_in + gq) / V)^2 goes to part[blockIdx.x].
__global__ void __launch_bounds__(kBS) k_adj_rk(const BlockDesc *blks, int b, const double *lam0, const double *qbar,
                         const double *gq, const double *dtv, const double *V, double alpha,
                         double *lam, double *part) {
    const BlockDesc &B = blks[b];
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (t < plane) {
        const double iv = 1.0 / V[B.cell_off + t];
        for (int n = 0; n < B.ns; ++n) {
            const double f = alpha * dtv[B.q_off / 4 + (int64_t)n * plane + t];
            for (int v = 0; v < 4; ++v) {
                const int64_t o = B.q_off + ((int64_t)n * 4 + v) * plane + t;
                const double r = qbar[o] + gq[o];
                lam[o] = lam0[o] - f * r;
                acc += (r * iv) * (r * iv);
            }
        }
    }
    if (!part) return;
    __shared__ double red[kBS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBS) k_adj_norm(const double *part, int64_t n, double inv_count, double *out) {
    __shared__ double red[kBS];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += kBS) acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0] * inv_count);
}

template <class T>
int upload(T **d, const std::vector<T> &h) {
    *d = nullptr;
    int rc = check_hip(hipMalloc((void **)d, sizeof(T) * std::max<size_t>(1, h.size())), "adjoint alloc");
    if (rc) return rc;
    if (h.empty()) return HB_OK;
    return check_hip(hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice), "upload");
}

int adjoint_setup(hb_grid *g) {
    if (g->AFI_d) return HB_OK;
    // inverse ghost map (CSR over global cells) and far-field ghost lists
    std::vector<std::vector<int>> eb(g->n_cells), ep(g->n_cells), em(g->n_cells);
    std::vector<int> ffptr(1, 0), ffp, ffm;
    std::vector<int8_t> ffc;
    g->ffc_off.assign(g->nblocks, 0);
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &K = g->blk[b];
        const int we = K.ni + 4;
        g->ffc_off[b] = (int64_t)ffc.size();
        ffc.resize(ffc.size() + (size_t)we * (K.nj + 4), 0);
        for (int je = 0; je < K.nj + 4; ++je)
            for (int ie = 0; ie < we; ++ie) {
                const int i = ie - 2, j = je - 2;
                if (i >= 0 && i < K.ni && j >= 0 && j < K.nj) continue;
                const GSrc s = ghost_src(g->blk, g->segs, b, i, j);
                const int p = je * we + ie;
                if (s.cell) {
                    const BlockDesc &S = g->blk[s.b];
                    const int64_t gc = S.cell_off + (int64_t)s.j * S.ni + s.i;
                    eb[gc].push_back(b);
                    ep[gc].push_back(p);
                    em[gc].push_back(s.mir);
                } else {
                    ffp.push_back(p);
                    ffm.push_back(s.mir);
                    ffc[g->ffc_off[b] + p] = s.mir ? -1 : 1;
                }
            }
        ffptr.push_back((int)ffp.size());
    }
    std::vector<int> fptr(g->n_cells + 1, 0), fb, fp, fm;
    for (int64_t c = 0; c < g->n_cells; ++c) {
        fptr[c + 1] = fptr[c] + (int)eb[c].size();
        fb.insert(fb.end(), eb[c].begin(), eb[c].end());
        fp.insert(fp.end(), ep[c].begin(), ep[c].end());
        fm.insert(fm.end(), em[c].begin(), em[c].end());
    }
    int rc = upload(&g->fold_ptr_d, fptr);
    rc = rc ? rc : upload(&g->fold_b_d, fb);
    rc = rc ? rc : upload(&g->fold_p_d, fp);
    rc = rc ? rc : upload(&g->fold_m_d, fm);
    rc = rc ? rc : upload(&g->ff_ptr_d, ffptr);
    rc = rc ? rc : upload(&g->ff_p_d, ffp);
    rc = rc ? rc : upload(&g->ff_m_d, ffm);
    rc = rc ? rc : upload(&g->ffc_d, ffc);
    if (rc) return rc;
    auto alloc = [&](double **p, int64_t n) {
        return check_hip(hipMalloc((void **)p, sizeof(double) * std::max<int64_t>(1, n)), "adjoint alloc");
    };
    rc = alloc(&g->AFI_d, g->n_afi);
    rc = rc ? rc : alloc(&g->AFJ_d, g->n_afj);
    rc = rc ? rc : alloc(&g->NB_d, g->n_nodeq);
    rc = rc ? rc : alloc(&g->WBext_d, g->n_ext);
    // alpha0 partials: one per workgroup of k_adj_alpha, blocks in order
    g->apart_off.assign(g->nblocks, 0);
    int np = 0;
    for (int b = 0; b < g->nblocks; ++b) {
        g->apart_off[b] = np;
        np += (int)std::max<unsigned>(1u, nblk((int64_t)(ffptr[b + 1] - ffptr[b]) * g->blk[b].ns));
    }
    g->n_apart = np;
    rc = rc ? rc : alloc(&g->adj_part_d, np + 1);
    // alpha0 partials of the residual adjoint: one per cell-adjoint workgroup
    g->cpart_off.assign(g->nblocks, 0);
    int64_t nc = 0;
    for (int b = 0; b < g->nblocks; ++b) {
        g->cpart_off[b] = nc;
        nc += nblk((int64_t)(g->blk[b].ni + 4) * (g->blk[b].nj + 4) * g->blk[b].ns);
    }
    g->n_cpart = nc;
    rc = rc ? rc : alloc(&g->cpart_d, nc);
    rc = rc ? rc : alloc(&g->geo_d, 6 * (g->n_fi + g->n_fj));
    rc = rc ? rc : alloc(&g->mb_d, (g->n_afi + g->n_afj) / kAF * 2);
    rc = rc ? rc : alloc(&g->vb_d, (int64_t)kMaxNs * g->n_cells);
    rc = rc ? rc : alloc(&g->cf_adj_d, g->n_forces);
    if (!rc && !g->ext_d) rc = alloc(&g->ext_adj_d, g->n_ext);
    return rc;
}

// fold one thread per cell and snapshot when one per cell would leave most
// CUs idle (fewer than 256 workgroups)
bool fold_per_snap(const BlockDesc &B) { return (int64_t)B.ni * B.nj < 256 * (int64_t)kBS; }

// XCD-aware order for the face and cell kernels of a block with fewer than
// 2^22 items: measured 3-5% faster adjoint at 256x128 N_H = 2, 1-3% slower
// at 1024x512 N_H = 4, which keeps the launch order
int adj_xcd(int64_t n) { return n < ((int64_t)1 << 22); }
unsigned adj_grid(int64_t n) { return adj_xcd(n) ? xcd_grid(n) : nblk(n); }

typedef void (*FaceKernel)(const BlockDesc *, int, const double *, const double *, const double *,
                           const double *, const double *, const double *, Consts, double *, double *,
                           int64_t, int, Motion, const double *, double *, double *);

FaceKernel face_kernel(bool nt, bool mv, bool geo) {
    if (geo) {
        if (mv) return nt ? k_adj_faces<true, true, true> : k_adj_faces<false, true, true>;
        return nt ? k_adj_faces<true, false, true> : k_adj_faces<false, false, true>;
    }
    if (mv) return nt ? k_adj_faces<true, true, false> : k_adj_faces<false, true, false>;
    return nt ? k_adj_faces<true, false, false> : k_adj_faces<false, false, false>;
}

void launch_wall_motion(hb_grid *g, double *xybar, hipStream_t s) {
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_adj_wall_motion, dim3(nblk((int64_t)4 * (B.ni + 4) * B.ns)), dim3(kBS), 0, s,
                           g->blk_d, b, g->WBext_d, g->motion, xybar);
    }
}

void launch_alpha(hb_grid *g, hipStream_t s) {
    for (int b = 0; b < g->nblocks; ++b) {
        const int next = b + 1 < g->nblocks ? g->apart_off[b + 1] : g->n_apart;
        hipLaunchKernelGGL(k_adj_alpha, dim3(next - g->apart_off[b]), dim3(kBS), 0, s, g->blk_d, b,
                           g->WBext_d, g->ff_ptr_d, g->ff_p_d, g->ff_m_d, g->ffw_d,
                           g->adj_part_d + g->apart_off[b]);
    }
}

}  // namespace

int launch_residual_adjoint(hb_grid *g, const double *q, const double *rbar, double *qbar,
                            double *xybar, double *flowbar, hipStream_t s, bool fill) {
    int rc = adjoint_setup(g);
    if (rc) return rc;
    double *ext = g->ext_d ? g->ext_d : g->ext_adj_d;
    const Consts c = g->consts;
    for (int b = 0; b < g->nblocks && fill; ++b) {
        rc = plain_ghost_fill(g, b, q, ext, s);
        if (rc) return rc;
    }
    // the node (or cell) kernels clear xybar; the cell kernels leave the alpha0
    // partials, which the first fold launch sums; on a moving grid the face
    // kernels store the midpoint adjoints for xybar
    double *mbi = (g->motion.tab && xybar) ? g->mb_d : nullptr;
    double *mbj = mbi ? g->mb_d + g->n_afi / kAF * 2 : nullptr;
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        const int64_t nI = (int64_t)(B.ni + 1) * B.nj * B.ns, nJ = (int64_t)B.ni * (B.nj + 1) * B.ns;
        const bool nt = (double)kAF * 8.0 * (double)(nI + nJ) > 256.0 * (1 << 20);
        const int64_t nw = 256 * (((nI > nJ ? nI : nJ) + 127) / 128);
        const bool mv = g->motion.tab != nullptr;
        hipLaunchKernelGGL(face_kernel(nt, mv, xybar != nullptr),
                           dim3(adj_grid(nw)),
                           dim3(kBS), 0, s, g->blk_d, b, ext, g->SI_d, g->dI_d, g->SJ_d, g->dJ_d,
                           rbar, c, g->AFI_d, g->AFJ_d, nI, adj_xcd(nw), g->motion, g->xy_d, mbi, mbj);
        // records that stay in the last-level cache: the cell kernel sums
        // the node adjoints itself (one launch fewer); else the node kernel
        const int64_t ne = (int64_t)(B.ni + 4) * (B.nj + 4) * B.ns;
        if (nt)
            hipLaunchKernelGGL(k_adj_nodes, dim3(nblk((int64_t)(B.ni + 1) * (B.nj + 1) * B.ns)), dim3(kBS), 0,
                               s, g->blk_d, b, g->AFI_d, g->AFJ_d, g->NB_d, xybar);
        hipLaunchKernelGGL(nt ? k_adj_cells<false> : k_adj_cells<true>, dim3(adj_grid(ne)), dim3(kBS), 0,
                           s, g->blk_d, b, ext, g->AFI_d, g->AFJ_d, g->NB_d, c, g->WBext_d,
                           g->ffc_d + g->ffc_off[b], g->ffw_d,
                           flowbar ? g->cpart_d + g->cpart_off[b] : (double *)nullptr, adj_xcd(ne),
                           nt ? (double *)nullptr : xybar);
    }
    // every block's extended adjoints exist before any fold (cuts read
    // neighbours); with xybar each fold launch also runs its block's
    // coordinate face step
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        const int64_t nc = (int64_t)B.ni * B.nj;
        const bool ps = fold_per_snap(B);
        const unsigned nf = ps ? (unsigned)((nc + kBS / B.ns - 1) / (kBS / B.ns)) : nblk(nc);
        XyStep xs{};
        if (xybar) {
            const int64_t nI = (int64_t)(B.ni + 1) * B.nj, nJ = (int64_t)B.ni * (B.nj + 1);
            xs = XyStep{g->AFI_d, g->AFJ_d, mbi, mbj, g->xy_d, g->C_d, xybar, g->geo_d,
                        g->n_fi, g->n_fj, nI, nI + nJ, nf};
        }
        const dim3 grid(nf + (xybar ? nblk(xs.n) : 0u));
        if (ps)
            hipLaunchKernelGGL(k_adj_fold<true>, grid, dim3(kBS), 0, s, g->blk_d, b,
                               q, rbar, g->WBext_d, g->fold_ptr_d, g->fold_b_d, g->fold_p_d, g->fold_m_d,
                               g->V_d, g->D_d, c, qbar, g->cpart_d, g->n_cpart,
                               b == 0 ? flowbar : (double *)nullptr, xybar ? g->vb_d : (double *)nullptr,
                               g->n_cells, xs);
        else
            hipLaunchKernelGGL(k_adj_fold<false>, grid, dim3(kBS), 0, s, g->blk_d, b,
                               q, rbar, g->WBext_d, g->fold_ptr_d, g->fold_b_d, g->fold_p_d, g->fold_m_d,
                               g->V_d, g->D_d, c, qbar, g->cpart_d, g->n_cpart,
                               b == 0 ? flowbar : (double *)nullptr, xybar ? g->vb_d : (double *)nullptr,
                               g->n_cells, xs);
    }
    if (xybar) {
        // every block's face step is done before any node gather (its
        // ghost-side atomics may reach a neighbour's nodes)
        if (g->motion.tab) launch_wall_motion(g, xybar, s);
        for (int b = 0; b < g->nblocks; ++b) {
            const BlockDesc &B = g->blk[b];
            hipLaunchKernelGGL(k_adj_xy_nodes, dim3(nblk((int64_t)4 * (B.ni + 1) * (B.nj + 1))), dim3(kBS), 0,
                               s, g->blk_d, b, g->geo_d, g->n_fi, g->n_fj, g->vb_d,
                               fold_per_snap(B) ? B.ns : 1, g->n_cells, g->xy_d, mbi != nullptr, xybar);
        }
    }
    return check_hip(hipGetLastError(), "adjoint launch");
}

// Adjoint pseudo-time iteration for (dR*/dQ)^T lam = -gq at a fixed state q:
// the forward multistage scheme with the same frozen local steps,
//   lam(k) = lam(0) - alpha_k (dtau/V) (J^T lam(k-1) + gq),
// whose iteration matrix has the eigenvalues of the forward linearisation.
// resnorm[it] = RMS over cells, snapshots and variables of (J^T lam + gq)/V
// at the first stage.
int adjoint_prepare(hb_grid *g, bool iterate) {
    int rc = adjoint_setup(g);
    if (rc || !iterate || g->it_lam0_d) return rc;
    int64_t np = 0;
    for (int b = 0; b < g->nblocks; ++b) np += nblk((int64_t)g->blk[b].ni * g->blk[b].nj);
    g->n_it_part = np;
    auto alloc = [&](double **p, int64_t n) {
        return check_hip(hipMalloc((void **)p, sizeof(double) * std::max<int64_t>(1, n)),
                         "adjoint iteration alloc");
    };
    rc = alloc(&g->it_lam0_d, g->n_state);
    rc = rc ? rc : alloc(&g->it_qbar_d, g->n_state);
    rc = rc ? rc : alloc(&g->it_dtv_d, g->n_state / 4);
    rc = rc ? rc : alloc(&g->it_part_d, np);
    return rc;
}

int launch_adjoint_iterate(hb_grid *g, const double *q, double *lam, const double *gq,
                           int n_iter, double *resnorm, hipStream_t s) {
    int rc = adjoint_prepare(g, true);
    if (rc) return rc;
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_adj_dtv, dim3(nblk((int64_t)B.ni * B.nj)), dim3(kBS), 0, s, g->blk_d, b,
                           q, g->SI_d, g->SJ_d, g->V_d, g->consts, g->it_dtv_d, g->motion, g->C_d);
    }
    // q is fixed over the iteration: its ghost-extended copy is filled once
    double *ext = g->ext_d ? g->ext_d : g->ext_adj_d;
    for (int b = 0; b < g->nblocks; ++b) {
        rc = plain_ghost_fill(g, b, q, ext, s);
        if (rc) return rc;
    }
    const int ns = g->solver.n_stages;
    for (int it = 0; it < n_iter; ++it) {
        rc = check_hip(hipMemcpyAsync(g->it_lam0_d, lam, sizeof(double) * g->n_state,
                                      hipMemcpyDeviceToDevice, s), "lambda copy");
        if (rc) return rc;
        for (int k = 0; k < ns; ++k) {
            rc = launch_residual_adjoint(g, q, lam, g->it_qbar_d, nullptr, nullptr, s, false);
            if (rc) return rc;
            int64_t po = 0;
            const bool norm = (k == 0) && resnorm;
            for (int b = 0; b < g->nblocks; ++b) {
                const BlockDesc &B = g->blk[b];
                const unsigned nb = nblk((int64_t)B.ni * B.nj);
                hipLaunchKernelGGL(k_adj_rk, dim3(nb), dim3(kBS), 0, s, g->blk_d, b, g->it_lam0_d,
                                   g->it_qbar_d, gq, g->it_dtv_d, g->V_d, g->solver.rk_alpha[k], lam,
                                   norm ? g->it_part_d + po : nullptr);
                po += nb;
            }
            if (norm)
                hipLaunchKernelGGL(k_adj_norm, dim3(1), dim3(kBS), 0, s, g->it_part_d, g->n_it_part,
                                   1.0 / (double)g->n_state, resnorm + it);
        }
    }
    return check_hip(hipGetLastError(), "adjoint iteration launch");
}

int launch_forces_adjoint(hb_grid *g, const double *q, const double *cfbar, double *qbar,
                          double *xybar, double *flowbar, hipStream_t s) {
    int rc = adjoint_setup(g);
    if (rc) return rc;
    double *ext = g->ext_d ? g->ext_d : g->ext_adj_d;
    const Consts c = g->consts;
    const double qinf = 0.5 * g->flow.mach * g->flow.mach, L = g->flow.l_ref;
    const ForceAdj fa{cfbar, g->body_off_d, cos(g->flow.alpha0), sin(g->flow.alpha0), qinf * L,
                      qinf * L * L, g->flow.x_mom, g->flow.y_mom};
    if (xybar)
        hipLaunchKernelGGL(k_zero, dim3(nblk(2 * g->n_nodes)), dim3(kBS), 0, s, xybar, 2 * g->n_nodes);
    hipLaunchKernelGGL(k_zero, dim3(nblk(g->n_afi)), dim3(kBS), 0, s, g->AFI_d, g->n_afi);
    hipLaunchKernelGGL(k_zero, dim3(nblk(g->n_afj)), dim3(kBS), 0, s, g->AFJ_d, g->n_afj);
    for (int b = 0; b < g->nblocks; ++b) {
        rc = plain_ghost_fill(g, b, q, ext, s);
        if (rc) return rc;
    }
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_adj_force_face, dim3(nblk((int64_t)B.ni * B.ns)), dim3(kBS), 0, s,
                           g->blk_d, b, ext, g->xy_d, g->SJ_d, g->dJ_d, fa, c, g->AFJ_d, xybar, g->motion);
        hipLaunchKernelGGL(k_adj_nodes, dim3(nblk((int64_t)(B.ni + 1) * (B.nj + 1) * B.ns)), dim3(kBS), 0,
                           s, g->blk_d, b, g->AFI_d, g->AFJ_d, g->NB_d, (double *)nullptr);
        hipLaunchKernelGGL(k_adj_cells<false>, dim3(adj_grid((int64_t)(B.ni + 4) * (B.nj + 4) * B.ns)), dim3(kBS), 0,
                           s, g->blk_d, b, ext, g->AFI_d, g->AFJ_d, g->NB_d, c, g->WBext_d,
                           g->ffc_d + g->ffc_off[b], g->ffw_d, (double *)nullptr,
                           adj_xcd((int64_t)(B.ni + 4) * (B.nj + 4) * B.ns), (double *)nullptr);
    }
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        hipLaunchKernelGGL(k_adj_fold<false>, dim3(nblk((int64_t)B.ni * B.nj)), dim3(kBS), 0, s, g->blk_d, b,
                           q, (const double *)nullptr, g->WBext_d, g->fold_ptr_d, g->fold_b_d,
                           g->fold_p_d, g->fold_m_d, g->V_d, g->D_d, c, qbar,
                           (const double *)nullptr, (int64_t)0, (double *)nullptr, (double *)nullptr,
                           (int64_t)0, XyStep{});
    }
    if (flowbar) {
        launch_alpha(g, s);
        rc = launch_forces(g, q, g->cf_adj_d, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_adj_force_axes, dim3(1), dim3(kBS), 0, s, g->cf_adj_d, cfbar,
                           (int)(g->n_forces / 3), g->adj_part_d + g->n_apart);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, g->adj_part_d, g->n_apart + 1, flowbar);
    }
    if (xybar) {
        if (g->motion.tab) launch_wall_motion(g, xybar, s);
        for (int b = 0; b < g->nblocks; ++b) {
            const BlockDesc &B = g->blk[b];
            const int64_t nI = (int64_t)(B.ni + 1) * B.nj, nJ = (int64_t)B.ni * (B.nj + 1);
            hipLaunchKernelGGL(k_adj_xy, dim3(nblk(nI + nJ)), dim3(kBS), 0, s, g->blk_d, b, g->AFI_d,
                               g->AFJ_d, (const double *)nullptr, (const double *)nullptr, g->xy_d,
                               g->C_d, xybar, g->geo_d, g->n_fi, g->n_fj, nI);
            hipLaunchKernelGGL(k_adj_xy_nodes, dim3(nblk((int64_t)4 * (B.ni + 1) * (B.nj + 1))), dim3(kBS), 0,
                               s, g->blk_d, b, g->geo_d, g->n_fi, g->n_fj, (const double *)nullptr, 0,
                               (int64_t)0, g->xy_d, 0, xybar);
        }
    }
    return check_hip(hipGetLastError(), "forces adjoint launch");
}

}  // namespace hb
