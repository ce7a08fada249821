// Device functions shared by the kernels of libhb: ghost resolution,
// MUSCL / van Albada reconstruction, Roe flux, diamond-path viscous flux,
// local time step.  Templated on the arithmetic type T (double or float).
//
// Face geometry: S is the face normal scaled by the face length, pointing
// from cell L to cell R; d = (centre of R) - (centre of L).  The edge of an
// i-face runs from node (i, j) to node (i, j+1); that of a j-face from node
// (i+1, j) to node (i, j), so that in both cases rot(end - start) = S with
// rot(x, y) = (y, -x).
#pragma once

#include <hip/hip_runtime.h>

#include "hb_internal.hpp"

namespace hb {

template <class T>
struct W4 {
    T r, u, v, p;
};

// Values that are the same in every lane (block descriptors, tile table
// entries) are read with ordinary loads; readfirstlane makes that known to
// the compiler, which then keeps them, and addresses built from them, in
// scalar registers.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Global load/store at (uniform base)[lane index] with a 32-bit byte offset,
// so that the address is a scalar base plus one 32-bit VGPR (valid while
// idx * sizeof(T) < 2^32: in-plane indices of one block).
template <class T>
__device__ __forceinline__ T ldg(const T *base, unsigned idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stg(T *base, unsigned idx, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (unsigned)sizeof(T)) = v;
}

// Reciprocal and square root: exact IEEE operations in FP64; in FP32 the
// hardware v_rcp_f32 / v_sqrt_f32 (1 ulp), well inside the FP32 budget
// and much shorter than the correctly rounded sequences.
template <class T>
__device__ __forceinline__ T frcp(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <class T>
__device__ __forceinline__ T fsqrt(T x) { return sqrt(x); }
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

template <class T>
__device__ __forceinline__ W4<T> prim_from_cons(T q0, T q1, T q2, T q3, T gm1) {
    W4<T> w;
    T ir = T(1) / q0;
    w.r = q0;
    w.u = q1 * ir;
    w.v = q2 * ir;
    w.p = gm1 * (q3 - T(0.5) * q0 * (w.u * w.u + w.v * w.v));
    return w;
}

template <class T>
__device__ __forceinline__ W4<T> mirror(W4<T> w) {
    w.u = -w.u;
    w.v = -w.v;
    return w;
}

// ---------------------------------------------------------------------------
// Ghost resolution.  A cell index (i, j) with i in [-2, ni+2), j in [-2, nj+2)
// is mapped to a value: interior cells are read; outside, the i sides are
// resolved first, then the j sides (which defines the corner ghosts); a cut
// continues in the glued block (cut_cell), whose own rules then apply to
// what is still outside it; on a partly glued side the cells no segment
// covers follow the side's rest kind (wall or far field).  `cell` is a functor (block, i, j) -> value
// reading an interior cell of any block; `ff(b)` returns the block's free
// stream of the current snapshot and `mir` the no-slip wall image of a
// value (applied once per wall met, so two walls cancel); `onwall(block,
// side, position)` is told each wall face the resolution mirrors at.
// ---------------------------------------------------------------------------
struct NoWall {
    __device__ void operator()(int, int, int) const {}
};

template <class V, class Interior, class FF, class Mir, class Wall = NoWall>
__device__ __forceinline__ V value_ij(const BlockDesc *blks, int b, int i, int j,
                                      const Interior &cell, const FF &ff, const Mir &mir,
                                      const Wall &onwall = Wall()) {
    bool m = false;
    for (int hop = 0; hop < kGhostHops; ++hop) {
        const BlockDesc &B = blks[b];
        if (i < 0 || i >= B.ni) {
            const int side = i < 0 ? 0 : 1;
            const int k = i < 0 ? -1 - i : i - B.ni;
            const int kind = B.bc[side];
            if (kind == HB_BC_PERIODIC) {
                i = i < 0 ? i + B.ni : i - B.ni;
            } else if (glued_at(B, B.segs, side, j)) {
                int a, ia, ja;
                cut_cell(blks, B.segs, b, side, k, j, &a, &ia, &ja);
                b = a;
                i = ia;
                j = ja;
            } else if (kind == HB_BC_WALL || (kind == HB_BC_CUT && B.rest[side] == HB_BC_WALL)) {
                onwall(b, side, j);
                i = side == 0 ? k : B.ni - 1 - k;
                m = !m;
            } else {
                const V f = ff(b);
                return m ? mir(f) : f;
            }
            continue;
        }
        if (j < 0 || j >= B.nj) {
            const int side = j < 0 ? 2 : 3;
            const int k = j < 0 ? -1 - j : j - B.nj;
            const int kind = B.bc[side];
            if (kind == HB_BC_PERIODIC) {
                j = j < 0 ? j + B.nj : j - B.nj;
            } else if (kind == HB_BC_WAKECUT && (i < B.wake || i >= B.ni - B.wake)) {
                i = B.ni - 1 - i;
                j = k;
            } else if (glued_at(B, B.segs, side, i)) {
                int a, ia, ja;
                cut_cell(blks, B.segs, b, side, k, i, &a, &ia, &ja);
                b = a;
                i = ia;
                j = ja;
            } else if (kind == HB_BC_WALL || kind == HB_BC_WAKECUT ||
                       (kind == HB_BC_CUT && B.rest[side] == HB_BC_WALL)) {
                onwall(b, side, i);
                j = side == 2 ? k : B.nj - 1 - k;
                m = !m;
            } else {
                const V f = ff(b);
                return m ? mir(f) : f;
            }
            continue;
        }
        const V v = cell(b, i, j);
        return m ? mir(v) : v;
    }
    return ff(b);      // not reached: every ghost resolves (checked at grid creation)
}

// jmin face i of block B is a solid wall (carries loads): a WALL side, the
// profile part of a WAKECUT side, or a cell of a partly glued side with a
// wall rest that no segment covers.
__device__ __forceinline__ bool jmin_wall(const BlockDesc &B, int i) {
    if (B.bc[2] == HB_BC_WALL) return true;
    if (B.bc[2] == HB_BC_WAKECUT) return i >= B.wake && i < B.ni - B.wake;
    if (B.bc[2] == HB_BC_CUT && B.rest[2] == HB_BC_WALL) return cut_seg_at(B, B.segs, 2, i) < 0;
    return false;
}

// Load through a uniform base pointer and an unsigned 32-bit byte offset
// (scalar base plus one VGPR in the address).
template <class T>
__device__ __forceinline__ T ldgb(const T *base, unsigned byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Wall image of full primitives.
template <class T>
struct MirrorFull {
    __device__ W4<T> operator()(W4<T> w) const { return mirror(w); }
};

// ---------------------------------------------------------------------------
// Reconstruction
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T van_albada(T a, T b, T eps) {
    return (a + b) * (a * b + eps) * frcp(a * a + b * b + T(2) * eps);
}

// Face states between cells m1 and p0 of a grid line m2, m1, p0, p1.
template <class T>
__device__ __forceinline__ void muscl(const W4<T> &m2, const W4<T> &m1, const W4<T> &p0,
                                      const W4<T> &p1, T eps, W4<T> &L, W4<T> &R) {
    L.r = m1.r + T(0.5) * van_albada(m1.r - m2.r, p0.r - m1.r, eps);
    L.u = m1.u + T(0.5) * van_albada(m1.u - m2.u, p0.u - m1.u, eps);
    L.v = m1.v + T(0.5) * van_albada(m1.v - m2.v, p0.v - m1.v, eps);
    L.p = m1.p + T(0.5) * van_albada(m1.p - m2.p, p0.p - m1.p, eps);
    R.r = p0.r - T(0.5) * van_albada(p0.r - m1.r, p1.r - p0.r, eps);
    R.u = p0.u - T(0.5) * van_albada(p0.u - m1.u, p1.u - p0.u, eps);
    R.v = p0.v - T(0.5) * van_albada(p0.v - m1.v, p1.v - p0.v, eps);
    R.p = p0.p - T(0.5) * van_albada(p0.p - m1.p, p1.p - p0.p, eps);
}

// ---------------------------------------------------------------------------
// Roe flux on full primitive states, times the face length.
// ---------------------------------------------------------------------------
// A moving face passes vg = x_t . S (grid velocity times the length-weighted
// normal): the flux becomes F.n - (vg/|S|) U and the eigenvalues are taken
// relative to the face; vg = 0 is the fixed face.
template <class T>
__device__ __forceinline__ void roe_flux(const W4<T> &L, const W4<T> &R, T sx, T sy, T g,
                                         T delta_frac, T f[4], T vg = T(0)) {
    const T area = fsqrt(sx * sx + sy * sy);
    const T ia = frcp(area);
    const T nx = sx * ia, ny = sy * ia;
    const T gg = g / (g - T(1));
    const T hl = gg * L.p / L.r + T(0.5) * (L.u * L.u + L.v * L.v);
    const T hr = gg * R.p / R.r + T(0.5) * (R.u * R.u + R.v * R.v);
    const T sl = sqrt(L.r), sr = sqrt(R.r);
    const T iw = T(1) / (sl + sr);
    const T rt = sl * sr;
    const T ut = (sl * L.u + sr * R.u) * iw;
    const T vt = (sl * L.v + sr * R.v) * iw;
    const T ht = (sl * hl + sr * hr) * iw;
    const T q2t = ut * ut + vt * vt;
    const T ct = fsqrt((g - T(1)) * (ht - T(0.5) * q2t));
    const T qnt = ut * nx + vt * ny;
    const T qrel = qnt - vg * ia;
    const T dr = R.r - L.r, du = R.u - L.u, dv = R.v - L.v, dp = R.p - L.p;
    const T dqn = du * nx + dv * ny;
    const T ic2 = frcp(ct * ct);
    const T a1 = (dp - rt * ct * dqn) * T(0.5) * ic2;
    const T a4 = (dp + rt * ct * dqn) * T(0.5) * ic2;
    const T a2 = dr - dp * ic2;
    T l1 = fabs(qrel - ct), l4 = fabs(qrel + ct);
    const T l2 = fabs(qrel);
    if (delta_frac > T(0)) {
        const T d = delta_frac * ct;
        const T i2d = frcp(T(2) * d);
        if (l1 < d) l1 = (l1 * l1 + d * d) * i2d;
        if (l4 < d) l4 = (l4 * l4 + d * d) * i2d;
    }
    const T b1 = l1 * a1, b4 = l4 * a4, b2 = l2 * a2, bs = l2 * rt;
    const T d0 = b1 + b4 + b2;
    const T d1 = b1 * (ut - ct * nx) + b4 * (ut + ct * nx) + b2 * ut + bs * (du - nx * dqn);
    const T d2 = b1 * (vt - ct * ny) + b4 * (vt + ct * ny) + b2 * vt + bs * (dv - ny * dqn);
    const T d3 = b1 * (ht - qnt * ct) + b4 * (ht + qnt * ct) + b2 * (T(0.5) * q2t) +
                 bs * (ut * du + vt * dv - qnt * dqn);
    const T qnl = L.u * nx + L.v * ny, qnr = R.u * nx + R.v * ny;
    const T ml = L.r * qnl, mr = R.r * qnr;
    const T f0 = ml + mr;
    const T f1 = ml * L.u + mr * R.u + (L.p + R.p) * nx;
    const T f2 = ml * L.v + mr * R.v + (L.p + R.p) * ny;
    const T f3 = ml * hl + mr * hr;
    // conserved sums U_L + U_R (rho E = rho H - p) for the face-speed term
    const T u0 = L.r + R.r, u1 = L.r * L.u + R.r * R.u, u2 = L.r * L.v + R.r * R.v;
    const T u3 = L.r * hl - L.p + R.r * hr - R.p;
    f[0] = T(0.5) * (area * (f0 - d0) - vg * u0);
    f[1] = T(0.5) * (area * (f1 - d1) - vg * u1);
    f[2] = T(0.5) * (area * (f2 - d2) - vg * u2);
    f[3] = T(0.5) * (area * (f3 - d3) - vg * u3);
}

// ---------------------------------------------------------------------------
// Viscous flux (diamond path), times the face length.  Inputs are (u, v, T)
// triples at L, R and the edge end points P (start) and Q (end).
// grad phi = [(phi_R - phi_L) S + (phi_P - phi_Q) rot(d)] / (d . S).
// fv receives (tau.S)_x, (tau.S)_y and the energy term.
// ---------------------------------------------------------------------------
template <class T>
struct UVT {
    T u, v, t;
};

template <class T>
__device__ __forceinline__ void viscous_flux(const UVT<T> &L, const UVT<T> &R, const UVT<T> &P,
                                             const UVT<T> &Q, T sx, T sy, T dx, T dy, T mu,
                                             T kappa, T fv[3], T u0 = T(0), T v0 = T(0)) {
    const T iden = frcp(dx * sx + dy * sy);
    const T ax = sx * iden, ay = sy * iden;     // S / (d.S)
    const T bx = dy * iden, by = -dx * iden;    // rot(d) / (d.S)
    const T du = R.u - L.u, dv = R.v - L.v, dt = R.t - L.t;
    const T eu = P.u - Q.u, ev = P.v - Q.v, et = P.t - Q.t;
    const T ux = du * ax + eu * bx, uy = du * ay + eu * by;
    const T vx = dv * ax + ev * bx, vy = dv * ay + ev * by;
    const T tx = dt * ax + et * bx, ty = dt * ay + et * by;
    const T div = ux + vy;
    const T txx = mu * (T(2) * ux - T(2.0 / 3.0) * div);
    const T tyy = mu * (T(2) * vy - T(2.0 / 3.0) * div);
    const T txy = mu * (uy + vx);
    const T fx = txx * sx + txy * sy;
    const T fy = txy * sx + tyy * sy;
    // face velocity; (u0, v0) is added back when L and R hold perturbations
    const T uf = u0 + T(0.5) * (L.u + R.u), vf = v0 + T(0.5) * (L.v + R.v);
    fv[0] = fx;
    fv[1] = fy;
    fv[2] = uf * fx + vf * fy + kappa * (tx * sx + ty * sy);
}

template <class T>
__device__ __forceinline__ UVT<T> uvt(const W4<T> &w, T g) {
    return UVT<T>{w.u, w.v, g * w.p / w.r};
}

template <class T>
__device__ __forceinline__ UVT<T> avg4(const UVT<T> &a, const UVT<T> &b, const UVT<T> &c,
                                       const UVT<T> &d) {
    return UVT<T>{T(0.25) * (a.u + b.u + c.u + d.u), T(0.25) * (a.v + b.v + c.v + d.v),
                  T(0.25) * (a.t + b.t + c.t + d.t)};
}

// ---------------------------------------------------------------------------
// Local time step of one cell and snapshot.
// dtau = CFL V / (L_I + L_J + 4 (Lv_I + Lv_J) + V omega N_H)
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T local_dt(const W4<T> &w, T six, T siy, T sjx, T sjy, T V, T g,
                                      T mu_pr, T cfl, T omega_nh) {
    const T ir = frcp(w.r);
    const T c = fsqrt(g * w.p * ir);
    const T ai2 = six * six + siy * siy, aj2 = sjx * sjx + sjy * sjy;
    const T li = fabs(w.u * six + w.v * siy) + c * fsqrt(ai2);
    const T lj = fabs(w.u * sjx + w.v * sjy) + c * fsqrt(aj2);
    const T fac = fmax(T(4.0 / 3.0) * ir, g * ir) * mu_pr;
    const T lv = fac * (ai2 + aj2) * frcp(V);
    return cfl * V * frcp(li + lj + T(4) * lv + V * omega_nh);
}

// ---------------------------------------------------------------------------
// Perturbation form.  The fused kernels carry every snapshot's state as the
// deviation from that snapshot's free stream (rho_inf = 1, c_inf = 1,
// p_inf = 1/gamma, T_inf = 1).  Differences of O(1) quantities that cancel
// are then never formed in the working precision: the flux of a face is
// F(W) - F(W_inf) (the free-stream flux sums to zero over a closed cell),
// and the HB source is D (Q - Q_inf) + D Q_inf.  In exact arithmetic the
// results equal the plain form.
// ---------------------------------------------------------------------------
template <class T>
struct FS {
    T u, v, p, h;          // free-stream velocity, pressure, total enthalpy
    T gg;                  // gamma / (gamma - 1)
};

// conserved perturbation (d rho, d rho u, d rho v, d rho E) -> primitive
// perturbation (d rho, d u, d v, d p)
template <class T>
__device__ __forceinline__ W4<T> pert_prim(T dr, T dmx, T dmy, T de, T fu, T fv, T gm1) {
    const T rho = T(1) + dr;
    const T ir = frcp(rho);
    W4<T> w;
    w.r = dr;
    w.u = (dmx - fu * dr) * ir;
    w.v = (dmy - fv * dr) * ir;
    const T dk = w.u * (T(2) * fu + w.u) + w.v * (T(2) * fv + w.v);    // |u|^2 - |u_inf|^2
    w.p = gm1 * (de - T(0.5) * (dr * (fu * fu + fv * fv) + rho * dk));
    return w;
}

// pert_prim plus the temperature perturbation T - 1, sharing 1/rho
template <class T>
__device__ __forceinline__ W4<T> pert_prim_t(T dr, T dmx, T dmy, T de, T fu, T fv, T gm1, T g,
                                             T &tp) {
    const T rho = T(1) + dr;
    const T ir = frcp(rho);
    W4<T> w;
    w.r = dr;
    w.u = (dmx - fu * dr) * ir;
    w.v = (dmy - fv * dr) * ir;
    const T dk = w.u * (T(2) * fu + w.u) + w.v * (T(2) * fv + w.v);
    w.p = gm1 * (de - T(0.5) * (dr * (fu * fu + fv * fv) + rho * dk));
    tp = (g * w.p - w.r) * ir;
    return w;
}

// Face geometry in the form the batched kernel keeps in registers for a
// whole tile.  Diamond gradient: grad phi = (phi_R - phi_L) g1 n
// + (phi_P - phi_Q) b with g1 = |S| / (d.S) and b = rot(d) / (d.S).  With
// the velocity jump D = u_R - u_L and the edge difference e = u_P - u_Q the
// velocity gradient is G = g1 D n^T + e b^T, so that
//   (G + G^T) n - (2/3) tr(G) n
//       = g1 D + (b.n) e + [(1/3) g1 (D.n) - (2/3) (e.b)] n + (e.n) b
// and grad T . n = g1 (T_R - T_L) + (b.n) (T_P - T_Q).  The coefficients
// carry mu |S| (stress) and kappa |S| (heat flux).
template <class T>
struct FaceGeo {
    T nx, ny, ha;                 // unit normal, |S| / 2
    T mg1, mg3, mbn, mbx, mby;    // mu |S| x (g1, g1 / 3, b.n, b)
    T kg1, kbn;                   // kappa |S| x (g1, b.n)
};

template <class T>
__device__ __forceinline__ FaceGeo<T> face_geo(T sx, T sy, T dx, T dy, T mu, T kappa) {
    FaceGeo<T> f;
    const T area = fsqrt(sx * sx + sy * sy);
    const T ia = frcp(area);
    f.nx = sx * ia;
    f.ny = sy * ia;
    f.ha = T(0.5) * area;
    const T iden = frcp(dx * sx + dy * sy);
    const T g1 = area * iden;
    const T bx = dy * iden, by = -dx * iden;
    const T bn = bx * f.nx + by * f.ny;
    const T ma = mu * area, ka = kappa * area;
    f.mg1 = ma * g1;
    f.mg3 = f.mg1 * T(1.0 / 3.0);
    f.mbn = ma * bn;
    f.mbx = ma * bx;
    f.mby = ma * by;
    f.kg1 = ka * g1;
    f.kbn = ka * bn;
    return f;
}

// Viscous flux times the face length from FaceGeo (the same quantities as
// viscous_flux, in the face-normal form above); u0, v0 are added back to
// the face velocity when L and R hold perturbations.
template <class T>
__device__ __forceinline__ void viscous_flux_g(const UVT<T> &L, const UVT<T> &R, const UVT<T> &P,
                                               const UVT<T> &Q, const FaceGeo<T> &fg, T fv[3],
                                               T u0, T v0) {
    const T du = R.u - L.u, dv = R.v - L.v, dt = R.t - L.t;
    const T eu = P.u - Q.u, ev = P.v - Q.v, et = P.t - Q.t;
    const T dn = du * fg.nx + dv * fg.ny;
    const T en = eu * fg.nx + ev * fg.ny;
    const T c = fg.mg3 * dn - T(2.0 / 3.0) * (eu * fg.mbx + ev * fg.mby);
    const T fx = fg.mg1 * du + fg.mbn * eu + c * fg.nx + en * fg.mbx;
    const T fy = fg.mg1 * dv + fg.mbn * ev + c * fg.ny + en * fg.mby;
    const T uf = u0 + T(0.5) * (L.u + R.u), vf = v0 + T(0.5) * (L.v + R.v);
    fv[0] = fx;
    fv[1] = fy;
    fv[2] = uf * fx + vf * fy + (fg.kg1 * dt + fg.kbn * et);
}

// Roe flux minus the free-stream flux, times the face length (ha = |S| / 2);
// L and R are primitive perturbations of the same snapshot.  The Roe
// weights use r = sqrt(rho_R / rho_L) (sharing 1/rho_L with the enthalpy),
// so u~ = (u_L + r u_R) / (1 + r) and rho~ = rho_L r; 1/c~^2 gives the
// Harten width's reciprocal, h2d = 1 / (2 delta_frac).  The wave sum
//   sum_k |lambda_k| alpha_k r_k
// is regrouped around s14 = b1 + b4 and k = c~ (b4 - b1) - bs (dq_n):
//   d0 = s14 + b2,  d_u = u~ d0 + n_x k + bs du,  d_v = v~ d0 + n_y k + bs dv,
//   d_E = h~ s14 + q~_n k + b2 |u~|^2 / 2 + bs (u~ du + v~ dv).
// MV: a face moving with normal speed vgn (x_t . n): the eigenvalues are
// taken relative to the face, and -vgn (dU_L + dU_R) (conserved
// perturbations; the free-stream part -vgn 2 U_inf sums to zero around a
// cell, since the midpoint face speeds of a rigid motion do) joins the flux.
template <class T, bool MV = false>
__device__ __forceinline__ void roe_flux_pert_n(const W4<T> &L, const W4<T> &R, const FS<T> &f,
                                                T nx, T ny, T ha, T g, T delta_frac, T h2d,
                                                T out[4], T vgn = T(0)) {
    const T gg = f.gg;
    const T rl = T(1) + L.r, rr = T(1) + R.r;
    const T irl = frcp(rl), irr = frcp(rr);
    const T ul = f.u + L.u, vl = f.v + L.v, ur = f.u + R.u, vr = f.v + R.v;
    const T dhl = gg * (L.p - f.p * L.r) * irl +
                  T(0.5) * (L.u * (T(2) * f.u + L.u) + L.v * (T(2) * f.v + L.v));
    const T dhr = gg * (R.p - f.p * R.r) * irr +
                  T(0.5) * (R.u * (T(2) * f.u + R.u) + R.v * (T(2) * f.v + R.v));
    const T hl = f.h + dhl, hr = f.h + dhr;
    const T rw = fsqrt(rr * irl);
    const T iw = frcp(T(1) + rw);
    const T rt = rl * rw;
    const T ut = (ul + rw * ur) * iw;
    const T vt = (vl + rw * vr) * iw;
    const T ht = (hl + rw * hr) * iw;
    const T q2t = ut * ut + vt * vt;
    const T c2 = (g - T(1)) * (ht - T(0.5) * q2t);
    const T ct = fsqrt(c2);
    const T ic2 = frcp(c2);
    const T qnt = ut * nx + vt * ny;
    const T dr = R.r - L.r, du = R.u - L.u, dv = R.v - L.v, dp = R.p - L.p;
    const T dqn = du * nx + dv * ny;
    const T a1 = (dp - rt * ct * dqn) * T(0.5) * ic2;
    const T a4 = (dp + rt * ct * dqn) * T(0.5) * ic2;
    const T a2 = dr - dp * ic2;
    const T qrel = MV ? qnt - vgn : qnt;
    T l1 = fabs(qrel - ct), l4 = fabs(qrel + ct);
    const T l2 = fabs(qrel);
    if (delta_frac > T(0)) {
        const T d = delta_frac * ct;
        const T i2d = h2d * ct * ic2;           // 1 / (2 d)
        if (l1 < d) l1 = (l1 * l1 + d * d) * i2d;
        if (l4 < d) l4 = (l4 * l4 + d * d) * i2d;
    }
    const T b1 = l1 * a1, b4 = l4 * a4, b2 = l2 * a2, bs = l2 * rt;
    const T s14 = b1 + b4;
    const T d0 = s14 + b2;
    const T kw = ct * (b4 - b1) - bs * dqn;
    const T d1 = ut * d0 + nx * kw + bs * du;
    const T d2 = vt * d0 + ny * kw + bs * dv;
    const T d3 = ht * s14 + qnt * kw + b2 * (T(0.5) * q2t) + bs * (ut * du + vt * dv);
    const T qni = f.u * nx + f.v * ny;
    const T qpl = L.u * nx + L.v * ny, qpr = R.u * nx + R.v * ny;
    const T dml = L.r * (qni + qpl) + qpl;
    const T dmr = R.r * (qni + qpr) + qpr;
    const T f0 = dml + dmr;
    const T f1 = dml * ul + dmr * ur + qni * (L.u + R.u) + (L.p + R.p) * nx;
    const T f2 = dml * vl + dmr * vr + qni * (L.v + R.v) + (L.p + R.p) * ny;
    const T f3 = dml * hl + dmr * hr + qni * (dhl + dhr);
    if constexpr (MV) {
        // conserved perturbations: d(rho u) = d rho u + du (rho_inf = 1),
        // d(rho E) = d(rho H) - dp = d rho h_inf + rho dh - dp
        const T e0 = L.r + R.r;
        const T e1 = L.r * ul + L.u + R.r * ur + R.u;
        const T e2 = L.r * vl + L.v + R.r * vr + R.v;
        const T e3 = (L.r + R.r) * f.h + rl * dhl + rr * dhr - (L.p + R.p);
        out[0] = ha * (f0 - d0 - vgn * e0);
        out[1] = ha * (f1 - d1 - vgn * e1);
        out[2] = ha * (f2 - d2 - vgn * e2);
        out[3] = ha * (f3 - d3 - vgn * e3);
    } else {
        out[0] = ha * (f0 - d0);
        out[1] = ha * (f1 - d1);
        out[2] = ha * (f2 - d2);
        out[3] = ha * (f3 - d3);
    }
}

// ---------------------------------------------------------------------------
// Reverse mode (adjoint) of the FP64 face operators above.  Each *_rev
// function takes the forward inputs (recomputing what it needs) and the
// adjoint of the outputs, and ADDS the adjoints of the inputs.
// ---------------------------------------------------------------------------

// Reciprocal for the reverse-mode code: the hardware estimate v_rcp_f64
// refined by two Newton-Raphson steps r <- r + r (1 - x r), each of which
// squares the relative error; within an ulp or two of 1/x for the normal,
// finite arguments met here (not correctly rounded, unlike 1.0 / x, and
// about half its instructions).
__device__ __forceinline__ double adj_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// van Albada: returns v = VA(a, b) and its partial derivatives.
__device__ __forceinline__ double van_albada_d(double a, double b, double eps, double &da,
                                               double &db) {
    const double N = (a + b) * (a * b + eps);
    const double Dn = a * a + b * b + 2.0 * eps;
    const double iD = adj_rcp(Dn);
    const double v = N * iD;
    da = ((a * b + eps) + (a + b) * b - v * 2.0 * a) * iD;
    db = ((a * b + eps) + (a + b) * a - v * 2.0 * b) * iD;
    return v;
}

// MUSCL reverse for one variable: L = m1 + VA(m1-m2, p0-m1)/2,
// R = p0 - VA(p0-m1, p1-p0)/2.
__device__ __forceinline__ void muscl_rev1(double m2, double m1, double p0, double p1, double eps,
                                           double Lb, double Rb, double &m2b, double &m1b,
                                           double &p0b, double &p1b) {
    double da, db;
    van_albada_d(m1 - m2, p0 - m1, eps, da, db);
    const double va = 0.5 * Lb;
    m1b += Lb + va * (da - db);
    m2b -= va * da;
    p0b += va * db;
    double ea, eb;
    van_albada_d(p0 - m1, p1 - p0, eps, ea, eb);
    const double vb = -0.5 * Rb;
    p0b += Rb + vb * (ea - eb);
    m1b -= vb * ea;
    p1b += vb * eb;
}

// Roe flux reverse (full primitive states, FP64).  Fb: adjoint of the 4 flux
// components; adds to Lb, Rb (primitive adjoints) and sxb, syb.  vg: the face
// speed x_t . S of a moving face (roe_flux); with vgb non-NULL its adjoint is
// added to *vgb.
__device__ __forceinline__ void roe_flux_rev(const W4<double> &L, const W4<double> &R, double sx,
                                    double sy, double g, double delta_frac, const double Fb[4],
                                    W4<double> &Lb, W4<double> &Rb, double &sxb, double &syb,
                                    double vg = 0.0, double *vgb = nullptr) {
    // ---- forward recomputation
    const double area = sqrt(sx * sx + sy * sy);
    const double ia = adj_rcp(area);
    const double nx = sx * ia, ny = sy * ia;
    const double gg = g * adj_rcp(g - 1.0);
    const double irl = adj_rcp(L.r), irr = adj_rcp(R.r);
    const double hl = gg * L.p * irl + 0.5 * (L.u * L.u + L.v * L.v);
    const double hr = gg * R.p * irr + 0.5 * (R.u * R.u + R.v * R.v);
    const double sl = sqrt(L.r), sr = sqrt(R.r);
    const double iw = adj_rcp(sl + sr);
    const double rt = sl * sr;
    const double ut = (sl * L.u + sr * R.u) * iw;
    const double vt = (sl * L.v + sr * R.v) * iw;
    const double ht = (sl * hl + sr * hr) * iw;
    const double q2t = ut * ut + vt * vt;
    const double ct = sqrt((g - 1.0) * (ht - 0.5 * q2t));
    const double qnt = ut * nx + vt * ny;
    const double qrel = qnt - vg * ia;
    const double dr = R.r - L.r, du = R.u - L.u, dv = R.v - L.v, dp = R.p - L.p;
    const double dqn = du * nx + dv * ny;
    const double ict = adj_rcp(ct);
    const double ic2 = ict * ict;
    const double X = rt * ct * dqn;
    const double a1 = (dp - X) * 0.5 * ic2;
    const double a4 = (dp + X) * 0.5 * ic2;
    const double a2 = dr - dp * ic2;
    const double lam1 = qrel - ct, lam4 = qrel + ct;
    const double r1 = fabs(lam1), r4 = fabs(lam4);
    double l1 = r1, l4 = r4;
    const double dd = delta_frac * ct;
    const double idd = delta_frac > 0.0 ? adj_rcp(dd) : 0.0;
    const bool fix1 = delta_frac > 0.0 && r1 < dd, fix4 = delta_frac > 0.0 && r4 < dd;
    if (fix1) l1 = (r1 * r1 + dd * dd) * (0.5 * idd);
    if (fix4) l4 = (r4 * r4 + dd * dd) * (0.5 * idd);
    const double l2 = fabs(qrel);
    const double b1 = l1 * a1, b4 = l4 * a4, b2 = l2 * a2, bs = l2 * rt;
    const double d0 = b1 + b4 + b2;
    const double d1 = b1 * (ut - ct * nx) + b4 * (ut + ct * nx) + b2 * ut + bs * (du - nx * dqn);
    const double d2 = b1 * (vt - ct * ny) + b4 * (vt + ct * ny) + b2 * vt + bs * (dv - ny * dqn);
    const double d3 = b1 * (ht - qnt * ct) + b4 * (ht + qnt * ct) + b2 * (0.5 * q2t) +
                      bs * (ut * du + vt * dv - qnt * dqn);
    const double qnl = L.u * nx + L.v * ny, qnr = R.u * nx + R.v * ny;
    const double ml = L.r * qnl, mr = R.r * qnr;
    const double f0 = ml + mr;
    const double f1 = ml * L.u + mr * R.u + (L.p + R.p) * nx;
    const double f2 = ml * L.v + mr * R.v + (L.p + R.p) * ny;
    const double f3 = ml * hl + mr * hr;
    // ---- reverse sweep
    double areab = 0.5 * (Fb[0] * (f0 - d0) + Fb[1] * (f1 - d1) + Fb[2] * (f2 - d2) + Fb[3] * (f3 - d3));
    const double f0b = 0.5 * area * Fb[0], f1b = 0.5 * area * Fb[1];
    const double f2b = 0.5 * area * Fb[2], f3b = 0.5 * area * Fb[3];
    const double d0b = -f0b, d1b = -f1b, d2b = -f2b, d3b = -f3b;
    double nxb = 0.0, nyb = 0.0;
    double hlb = 0.0, hrb = 0.0;
    if (vgb)   // -vg (U_L + U_R) / 2
        *vgb -= 0.5 * (Fb[0] * (L.r + R.r) + Fb[1] * (L.r * L.u + R.r * R.u) +
                       Fb[2] * (L.r * L.v + R.r * R.v) + Fb[3] * (L.r * hl - L.p + R.r * hr - R.p));
    if (vg != 0.0) {
        // -vg (U_L + U_R) / 2 with U = (rho, rho u, rho v, rho H - p)
        const double u0 = -0.5 * vg * Fb[0], u1 = -0.5 * vg * Fb[1];
        const double u2 = -0.5 * vg * Fb[2], u3 = -0.5 * vg * Fb[3];
        Lb.r += u0 + u1 * L.u + u2 * L.v + u3 * hl;
        Rb.r += u0 + u1 * R.u + u2 * R.v + u3 * hr;
        Lb.u += u1 * L.r;
        Rb.u += u1 * R.r;
        Lb.v += u2 * L.r;
        Rb.v += u2 * R.r;
        Lb.p -= u3;
        Rb.p -= u3;
        hlb += u3 * L.r;
        hrb += u3 * R.r;
    }
    // central part
    const double mlb = f0b + f1b * L.u + f2b * L.v + f3b * hl;
    const double mrb = f0b + f1b * R.u + f2b * R.v + f3b * hr;
    Lb.u += f1b * ml;
    Rb.u += f1b * mr;
    Lb.v += f2b * ml;
    Rb.v += f2b * mr;
    Lb.p += f1b * nx + f2b * ny;
    Rb.p += f1b * nx + f2b * ny;
    nxb += f1b * (L.p + R.p);
    nyb += f2b * (L.p + R.p);
    hlb += f3b * ml;
    hrb += f3b * mr;
    Lb.r += mlb * qnl;
    Rb.r += mrb * qnr;
    const double qnlb = mlb * L.r, qnrb = mrb * R.r;
    Lb.u += qnlb * nx;
    Lb.v += qnlb * ny;
    Rb.u += qnrb * nx;
    Rb.v += qnrb * ny;
    nxb += qnlb * L.u + qnrb * R.u;
    nyb += qnlb * L.v + qnrb * R.v;
    // dissipation
    const double b1b = d0b + d1b * (ut - ct * nx) + d2b * (vt - ct * ny) + d3b * (ht - qnt * ct);
    const double b4b = d0b + d1b * (ut + ct * nx) + d2b * (vt + ct * ny) + d3b * (ht + qnt * ct);
    const double b2b = d0b + d1b * ut + d2b * vt + d3b * (0.5 * q2t);
    const double bsb = d1b * (du - nx * dqn) + d2b * (dv - ny * dqn) + d3b * (ut * du + vt * dv - qnt * dqn);
    const double bsum = b1 + b4 + b2;
    double utb = bsum * d1b + bs * du * d3b;
    double vtb = bsum * d2b + bs * dv * d3b;
    double ctb = (b4 - b1) * (d1b * nx + d2b * ny + d3b * qnt);
    nxb += d1b * (ct * (b4 - b1) - bs * dqn);
    nyb += d2b * (ct * (b4 - b1) - bs * dqn);
    double htb = d3b * (b1 + b4);
    double q2tb = d3b * 0.5 * b2;
    double qntb = d3b * (ct * (b4 - b1) - bs * dqn);
    double dub = d1b * bs + d3b * bs * ut;
    double dvb = d2b * bs + d3b * bs * vt;
    double dqnb = -bs * (d1b * nx + d2b * ny + d3b * qnt);
    const double l1b = b1b * a1, a1b = b1b * l1;
    const double l4b = b4b * a4, a4b = b4b * l4;
    const double l2b = b2b * a2 + bsb * rt;
    const double a2b = b2b * l2;
    double rtb = bsb * l2;
    // eigenvalues with Harten's fix
    double ddb = 0.0;
    double r1b = l1b, r4b = l4b;
    if (fix1) {
        r1b = l1b * r1 * idd;
        ddb += l1b * (dd * dd - r1 * r1) * (0.5 * idd * idd);
    }
    if (fix4) {
        r4b = l4b * r4 * idd;
        ddb += l4b * (dd * dd - r4 * r4) * (0.5 * idd * idd);
    }
    // d|x|/dx taken as sign(x) with sign(0) = 0, the average of the one-sided
    // derivatives (a wall face has q~_n = 0 exactly by symmetry)
    auto sgn = [](double x) { return (double)((x > 0.0) - (x < 0.0)); };
    const double lam1b = r1b * sgn(lam1);
    const double lam4b = r4b * sgn(lam4);
    const double qrelb = lam1b + lam4b + l2b * sgn(qrel);
    qntb += qrelb;
    areab += qrelb * vg * ia * ia;          // qrel = qnt - vg / |S|
    if (vgb) *vgb -= qrelb * ia;
    ctb += -lam1b + lam4b + delta_frac * ddb;
    // wave strengths
    double dpb = 0.5 * ic2 * (a1b + a4b) - ic2 * a2b;
    double drb = a2b;
    const double Xb = 0.5 * ic2 * (a4b - a1b);
    rtb += Xb * ct * dqn;
    ctb += Xb * rt * dqn;
    dqnb += Xb * rt * ct;
    const double ic2b = 0.5 * (dp - X) * a1b + 0.5 * (dp + X) * a4b - dp * a2b;
    ctb += ic2b * (-2.0 * ic2 * ict);
    // qnt, dqn
    utb += qntb * nx;
    vtb += qntb * ny;
    nxb += qntb * ut + dqnb * du;
    nyb += qntb * vt + dqnb * dv;
    dub += dqnb * nx;
    dvb += dqnb * ny;
    Rb.r += drb;
    Lb.r -= drb;
    Rb.u += dub;
    Lb.u -= dub;
    Rb.v += dvb;
    Lb.v -= dvb;
    Rb.p += dpb;
    Lb.p -= dpb;
    // ct = sqrt((g-1)(ht - q2t/2))
    const double c2b = ctb * (0.5 * ict);
    htb += (g - 1.0) * c2b;
    q2tb -= 0.5 * (g - 1.0) * c2b;
    utb += 2.0 * ut * q2tb;
    vtb += 2.0 * vt * q2tb;
    // Roe averages
    double slb = rtb * sr, srb = rtb * sl;
    Lb.u += utb * sl * iw;
    Rb.u += utb * sr * iw;
    slb += utb * (L.u - ut) * iw;
    srb += utb * (R.u - ut) * iw;
    Lb.v += vtb * sl * iw;
    Rb.v += vtb * sr * iw;
    slb += vtb * (L.v - vt) * iw;
    srb += vtb * (R.v - vt) * iw;
    hlb += htb * sl * iw;
    hrb += htb * sr * iw;
    slb += htb * (hl - ht) * iw;
    srb += htb * (hr - ht) * iw;
    // d sqrt(r) / dr = 1 / (2 sqrt(r)) = sqrt(r) / (2 r)
    Lb.r += slb * (0.5 * sl * irl);
    Rb.r += srb * (0.5 * sr * irr);
    // enthalpies
    Lb.p += hlb * gg * irl;
    Lb.r -= hlb * gg * L.p * irl * irl;
    Lb.u += hlb * L.u;
    Lb.v += hlb * L.v;
    Rb.p += hrb * gg * irr;
    Rb.r -= hrb * gg * R.p * irr * irr;
    Rb.u += hrb * R.u;
    Rb.v += hrb * R.v;
    // unit normal and face length
    sxb += (nxb * (1.0 - nx * nx) - nyb * nx * ny) * ia + areab * nx;
    syb += (nyb * (1.0 - ny * ny) - nxb * nx * ny) * ia + areab * ny;
}

// Viscous flux reverse.  fvb: adjoint of (fx, fy, fe); adds to the (u, v, T)
// adjoints at L, R, P (edge start), Q (edge end) and to S, d.
__device__ inline void viscous_flux_rev(const UVT<double> &L, const UVT<double> &R,
                                        const UVT<double> &P, const UVT<double> &Q, double sx,
                                        double sy, double dx, double dy, double mu, double kappa,
                                        const double fvb[3], UVT<double> &Lb, UVT<double> &Rb,
                                        UVT<double> &Pb, UVT<double> &Qb, double &sxb, double &syb,
                                        double &dxb, double &dyb) {
    const double den = dx * sx + dy * sy;
    const double iden = adj_rcp(den);
    const double ax = sx * iden, ay = sy * iden, bx = dy * iden, by = -dx * iden;
    const double du = R.u - L.u, dv = R.v - L.v, dt = R.t - L.t;
    const double eu = P.u - Q.u, ev = P.v - Q.v, et = P.t - Q.t;
    const double ux = du * ax + eu * bx, uy = du * ay + eu * by;
    const double vx = dv * ax + ev * bx, vy = dv * ay + ev * by;
    const double tx = dt * ax + et * bx, ty = dt * ay + et * by;
    const double div = ux + vy;
    const double txx = mu * (2.0 * ux - (2.0 / 3.0) * div);
    const double tyy = mu * (2.0 * vy - (2.0 / 3.0) * div);
    const double txy = mu * (uy + vx);
    const double fx = txx * sx + txy * sy;
    const double fy = txy * sx + tyy * sy;
    const double uf = 0.5 * (L.u + R.u), vf = 0.5 * (L.v + R.v);
    const double gx = fvb[0], gy = fvb[1], ge = fvb[2];
    // fe = uf fx + vf fy + kappa (tx sx + ty sy)
    const double ufb = ge * fx, vfb = ge * fy;
    const double fxb = gx + ge * uf, fyb = gy + ge * vf;
    const double txb = ge * kappa * sx, tyb = ge * kappa * sy;
    sxb += ge * kappa * tx;
    syb += ge * kappa * ty;
    // fx = txx sx + txy sy ; fy = txy sx + tyy sy
    const double txxb = fxb * sx, tyyb = fyb * sy, txyb = fxb * sy + fyb * sx;
    sxb += fxb * txx + fyb * txy;
    syb += fxb * txy + fyb * tyy;
    const double uxb = mu * ((4.0 / 3.0) * txxb - (2.0 / 3.0) * tyyb);
    const double vyb = mu * ((4.0 / 3.0) * tyyb - (2.0 / 3.0) * txxb);
    const double uyb = mu * txyb, vxb = mu * txyb;
    Lb.u += 0.5 * ufb;
    Rb.u += 0.5 * ufb;
    Lb.v += 0.5 * vfb;
    Rb.v += 0.5 * vfb;
    // gradients
    const double dub = uxb * ax + uyb * ay, eub = uxb * bx + uyb * by;
    const double dvb = vxb * ax + vyb * ay, evb = vxb * bx + vyb * by;
    const double dtb = txb * ax + tyb * ay, etb = txb * bx + tyb * by;
    const double axb = uxb * du + vxb * dv + txb * dt;
    const double ayb = uyb * du + vyb * dv + tyb * dt;
    const double bxb = uxb * eu + vxb * ev + txb * et;
    const double byb = uyb * eu + vyb * ev + tyb * et;
    Rb.u += dub;
    Lb.u -= dub;
    Rb.v += dvb;
    Lb.v -= dvb;
    Rb.t += dtb;
    Lb.t -= dtb;
    Pb.u += eub;
    Qb.u -= eub;
    Pb.v += evb;
    Qb.v -= evb;
    Pb.t += etb;
    Qb.t -= etb;
    // geometry
    const double idenb = axb * sx + ayb * sy + bxb * dy - byb * dx;
    sxb += axb * iden;
    syb += ayb * iden;
    dyb += bxb * iden;
    dxb -= byb * iden;
    const double denb = -iden * iden * idenb;
    dxb += denb * sx;
    sxb += denb * dx;
    dyb += denb * sy;
    syb += denb * dy;
}

// (u, v, T = gamma p / rho) adjoint -> primitive adjoint
__device__ __forceinline__ void uvt_rev(const W4<double> &w, const UVT<double> &b, double g,
                                        W4<double> &wb) {
    wb.u += b.u;
    wb.v += b.v;
    const double ir = adj_rcp(w.r);
    wb.p += b.t * g * ir;
    wb.r -= b.t * g * w.p * ir * ir;
}

// primitive adjoint -> conserved adjoint (rho, rho u, rho v, rho E)
__device__ __forceinline__ void prim_rev(const W4<double> &w, const W4<double> &wb, double gm1,
                                         double qb[4]) {
    const double ir = adj_rcp(w.r);
    qb[0] = wb.r - wb.u * w.u * ir - wb.v * w.v * ir + wb.p * gm1 * 0.5 * (w.u * w.u + w.v * w.v);
    qb[1] = wb.u * ir - wb.p * gm1 * w.u;
    qb[2] = wb.v * ir - wb.p * gm1 * w.v;
    qb[3] = wb.p * gm1;
}

}  // namespace hb
