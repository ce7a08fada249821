// Fused, batched residual / Runge-Kutta stage kernel.
//
// One launch per stage covers every block of the grid: the blocks are cut
// into tiles of 16 x 15 (or 32 x 7) cells (256 threads, one per cell of a
// 16 x 16 or 32 x 8 thread grid whose last row only helps), listed in a
// flat tile table sorted by snapshot count; the grid is one workgroup per
// tile or a persistent grid walking the table with a fixed stride (chosen
// by the autotuner, with an optional XCD-aware order).  Per tile:
//   A. every thread loads its cell's state for all N_s snapshots (as the
//      deviation from each snapshot's free stream);
//   B. the HB source D (Q - Q_inf) of the tile, a [cells x N_s] x [N_s x N_s]
//      product, runs on the matrix cores (FP32: v_mfma 16x16x4, operands
//      staged through LDS); FP64 tiles use FMA;
//   C. for each snapshot: the ghost-extended tile (2-cell halo; the sources
//      of a tile at a block side come from its host-built halo table) is
//      staged in LDS as primitive perturbations, node averages of (u, v, T)
//      are formed, each i- and j-face flux (MUSCL/van Albada + Roe,
//      diamond-path viscous) is computed once, and each cell sums its four
//      faces, adds V (D Q), and either writes R* or performs the Runge-Kutta
//      update in FP64 from the iteration's base state, with the local time
//      step formed from that base state by the iteration's first stage.
// The per-tile partial of sum (R*_rho / V)^2 goes to partials[tile]; a second
// kernel sums the partials in a fixed order (deterministic norm).
//
// This header holds the kernel and its launch templates; each combination of
// moving grid (MV) and 64-bit halo addressing (BIG) is instantiated in a
// translation unit of its own (hb_fused_k*.hip), the host side of the path
// (arguments, stage sequence, graphs, tile lists) is in hb_fused.hip.
#pragma once

#include "hb_device.hpp"

#include <algorithm>
#include <type_traits>

namespace hb {
namespace fk {

constexpr int kThreads = 256;
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <class T>
struct FusedArgs {
    const BlockDesc *blks;
    const Tile *tiles;
    const uint32_t *gtab;  // halo source tables of the tiles at block sides
    const uint64_t *gtab64;  // 64-bit addressing: the sources of the same entries (elements)
    int n_tiles;
    const double *q0;      // FP64 base state Q(0); also the stencil input of stage 1
    const T *sin;          // stencil input of later stages (perturbation form)
    T *sout;               // perturbation output of intermediate stages
    double *qout;          // FP64 output: R* (residual mode) or the new state (last stage)
    const T *SI, *dI, *SJ, *dJ, *V;
    const T *D;            // kNsPad x kNsPad per block
    const T *ffw;          // free-stream primitives per snapshot
    const T *dqinf;        // sum_m D[n][m] Q_inf(m) per snapshot
    const double *ffq;     // free-stream conserved variables per snapshot (FP64)
    double *partials;      // per tile
    T *dtau;               // local time step per cell-snapshot: written by the first stage
    int *status;
    T gamma, mu, kappa, mu_pr, cfl, delta, eps;
    double alpha;
    int norm;
    int dq_bytes;          // FP32: bytes of the LDS HB-source area before the scratch
    int xcd;               // XCD-aware renumbering: tiles per XCD chunk (0: off)
    T h2d;                 // 1 / (2 delta_frac) (Harten width), 0 without the fix
    // rigid grid motion (the moving-grid kernels only): per-snapshot table
    // of kMotionW doubles {cos theta, sin theta, theta_dot, h, h_dot, ..},
    // the pivot, the body-frame nodes and cell centres, and per ext cell of
    // the tiles at block sides the wall face of a moving no-slip image
    // (index of its first node's x in xy, and the node count of that
    // block; 0 = not a wall image)
    const double *mot;
    const double *xy;
    const double *C;
    const uint32_t *wtab;
    double xp, yp;
};

// Row stride (floats) of the LDS HB-source array DQs[N_s][4][cells].  (A
// stride of 258 with float2 write-back, which spreads the MFMA result rows
// over the LDS banks, measured 12% slower per stage.)
constexpr int kDqS = 256;

// Threads form a TI x TJ grid; the tile's output cells are TI x (TJ - 1):
// the last thread row only helps with loads, nodes and faces.  With
// TI = 16, TJ = 16 a tile has 255 i-faces and 256 j-faces, so each face
// pass is one round over the 256 threads (no wave gets a second round).
template <int TI, int TJ>
struct Geo {
    static constexpr int OJ = TJ - 1;                  // output rows
    static constexpr int WE = TI + 4;                  // ext row length
    static constexpr int EXT = (TI + 4) * (OJ + 4);
    static constexpr int NOD = (TI + 1) * (OJ + 1);
    static constexpr int NFI = (TI + 1) * OJ;
    static constexpr int NFJ = TI * (OJ + 1);
    static constexpr int NFMAX = NFI > NFJ ? NFI : NFJ;
    static constexpr int SCRATCH = 5 * EXT + 3 * NOD + 4 * NFMAX;   // elements
};

// Flux of one face of the tile (perturbation form, times the face length),
// written to F[v * fs + k].  IFACE: i-face k = fj*(TI+1) + fi between
// cells fi-1 and fi of row fj; else j-face k = fj*TI + fi between rows fj-1
// and fj of column fi.  Returns without writing for faces outside the block.
// Uniform per-tile data used by the face loops.
template <class T>
struct TileU {
    int ni, nj, i0, j0;
    const T *SI, *dI, *SJ, *dJ;      // block's face metrics
};

// Face k of the tile (the caller has checked that it lies in the block),
// geometry fg held in registers for the whole tile.
// MV: a moving face with normal speed vgn.
template <class T, int TI, int TJ, bool IFACE, bool MV>
__device__ __forceinline__ void face_flux(const FusedArgs<T> &a, int k, const T *P, const T *Nd,
                                          T *F, int fs, const FS<T> &f, const FaceGeo<T> &fg,
                                          T vgn) {
    using G = Geo<TI, TJ>;
    int e0, es, nA, nB;
    if constexpr (IFACE) {
        const int fi = k % (TI + 1), fj = k / (TI + 1);
        e0 = (fj + 2) * G::WE + fi;
        es = 1;
        nA = fj * (TI + 1) + fi;            // node (i, j): edge start
        nB = nA + (TI + 1);                 // node (i, j+1): edge end
    } else {
        const int fi = k % TI, fj = k / TI;
        e0 = fj * G::WE + fi + 2;
        es = G::WE;
        nB = fj * (TI + 1) + fi;            // node (i, j): edge end
        nA = nB + 1;                        // node (i+1, j): edge start
    }
    const int x0 = e0, x1 = e0 + es, x2 = e0 + 2 * es, x3 = e0 + 3 * es;
    const W4<T> m2{P[x0], P[G::EXT + x0], P[2 * G::EXT + x0], P[3 * G::EXT + x0]};
    const W4<T> m1{P[x1], P[G::EXT + x1], P[2 * G::EXT + x1], P[3 * G::EXT + x1]};
    const W4<T> p0{P[x2], P[G::EXT + x2], P[2 * G::EXT + x2], P[3 * G::EXT + x2]};
    const W4<T> p1{P[x3], P[G::EXT + x3], P[2 * G::EXT + x3], P[3 * G::EXT + x3]};
    W4<T> L, R;
    muscl(m2, m1, p0, p1, a.eps, L, R);
    T fl[4];
    roe_flux_pert_n<T, MV>(L, R, f, fg.nx, fg.ny, fg.ha, a.gamma, a.delta, a.h2d, fl, vgn);
    const UVT<T> uL{m1.u, m1.v, P[4 * G::EXT + x1]};
    const UVT<T> uR{p0.u, p0.v, P[4 * G::EXT + x2]};
    const UVT<T> na{Nd[nA], Nd[G::NOD + nA], Nd[2 * G::NOD + nA]};
    const UVT<T> nb{Nd[nB], Nd[G::NOD + nB], Nd[2 * G::NOD + nB]};
    T fv[3];
    viscous_flux_g(uL, uR, na, nb, fg, fv, f.u, f.v);
    F[k] = fl[0];
    F[fs + k] = fl[1] - fv[0];
    F[2 * fs + k] = fl[2] - fv[1];
    F[3 * fs + k] = fl[3] - fv[2];
}

// Scalar copy of the block descriptor fields the tile body uses.
struct BlockU {
    int ni, nj, snap_off, d_off;
    int64_t q_off, cell_off, node_off, fi_off, fj_off;
    double omega_nh;
};

// Face geometry of snapshot n on a rigidly rotated grid: the body-frame
// normal and diamond vector b turn with the grid (c, s = cos, sin theta_n);
// |S|, g1 and b.n do not change.
template <class T>
__device__ __forceinline__ FaceGeo<T> rotate_geo(const FaceGeo<T> &g, T c, T s) {
    FaceGeo<T> r = g;
    r.nx = c * g.nx - s * g.ny;
    r.ny = s * g.nx + c * g.ny;
    r.mbx = c * g.mbx - s * g.mby;
    r.mby = s * g.mbx + c * g.mby;
    return r;
}

// NS > 0: snapshot count fixed at compile time (FP64 tiles, whose HB source
// lives in registers); NS = 0: taken from the tile at run time (FP32 tiles:
// one body serves every snapshot count).  MV: the grid moves rigidly (ALE
// form: moving faces, moving no-slip wall images, the time step relative to
// the grid).  BIG: halo sources addressed by 64-bit element offsets (states
// of 4 GiB or more); otherwise by 32-bit byte offsets.
template <class T, int TI, int TJ, bool FIRST, int MODE, int NS, bool MV, bool BIG>
__device__ void tile_body(const FusedArgs<T> &a, const Tile &tl, int tile_id, unsigned char *smem,
                          int &bad) {
    using G = Geo<TI, TJ>;
    static_assert(TI * TJ == kThreads, "one thread per cell");
    // FP32: the HB source goes through the matrix cores and stays in LDS
    // (DQs, [N_s][4][cells]) for the whole snapshot loop; FP64: FMA, held in
    // registers.
    constexpr bool MF = std::is_same<T, float>::value;
    static_assert(MF || NS > 0, "FP64 tiles need a compile-time snapshot count");
    const int ns = NS > 0 ? NS : tl.ns;
    const BlockDesc &Bg = a.blks[tl.blk];
    BlockU B;
    B.ni = uni(Bg.ni);
    B.nj = uni(Bg.nj);
    B.snap_off = uni(Bg.snap_off);
    B.d_off = uni(Bg.d_off);
    B.q_off = uni(Bg.q_off);
    B.cell_off = uni(Bg.cell_off);
    B.node_off = MV ? uni(Bg.node_off) : 0;
    B.fi_off = uni(Bg.fi_off);
    B.fj_off = uni(Bg.fj_off);
    B.omega_nh = Bg.omega_nh;
    const int ni = B.ni, nj = B.nj;
    const TileU<T> tu{ni, nj, tl.i0, tl.j0, a.SI + 2 * B.fi_off, a.dI + 2 * B.fi_off,
                      a.SJ + 2 * B.fj_off, a.dJ + 2 * B.fj_off};
    const int tid = threadIdx.x;
    const int ti = tid % TI, tj = tid / TI;
    const int i = tl.i0 + ti, j = tl.j0 + tj;
    const bool valid = tj < G::OJ && i < ni && j < nj;
    // per-block offsets fit in 32 bits (ni nj <= 2^24, N_s <= 9).  Loads are
    // written as (uniform base pointer)[unsigned lane offset] so that the
    // address stays a scalar base plus one 32-bit VGPR offset.
    const int plane = ni * nj;
    const unsigned cidx = valid ? (unsigned)(j * ni + i) : 0u;
    const T g = a.gamma, gm1 = a.gamma - T(1);
    T *DQs = reinterpret_cast<T *>(smem);
    T *P = reinterpret_cast<T *>(smem + (MF ? a.dq_bytes : 0));   // [5][EXT]: rho', u', v', p', T'
    T *Nd = P + 5 * G::EXT;                                        // [3][NOD]: u', v', T' at nodes
    T *F = Nd + 3 * G::NOD;                                        // [4][NFMAX] i-faces
    // j-face fluxes: FP32 tiles write them into the HB-source slot of the
    // current snapshot (read into registers before); FP64 tiles, whose HB
    // source is in registers, have an area of their own after F
    T *FJ64 = F + 4 * G::NFMAX;
    // per-snapshot constants of the block, loaded once per tile:
    // Tf[n][8] = free-stream (u, v, p, -), D Q_inf (4); Td[n][4] = free-stream Q (FP64)
    T *Tf = F + (MF ? 4 : 8) * G::NFMAX;
    double *Td = reinterpret_cast<double *>(Tf + 8 * kMaxNs);
    // (loaded here into registers, written to LDS after the other set-up
    // loads have been issued)
    const bool wtf = tid < 8 * ns, wtd = tid >= 128 && tid < 128 + 4 * ns;
    T tfv = T(0);
    double tdv = 0.0;
    if (wtf) {
        const int n = tid >> 3, c = tid & 7;
        const int sn = 4 * (B.snap_off + n);
        if (c < 3) tfv = a.ffw[sn + 1 + c];
        else if (c > 3) tfv = a.dqinf[sn + c - 4];
    } else if (wtd) {
        tdv = a.ffq[4 * B.snap_off + tid - 128];
    }
    // halo source table entries of this thread's two ghost-extended cells
    // (tiles at block sides), issued first: the halo prefetch depends on them
    static_assert(Geo<TI, TJ>::EXT <= 2 * kThreads, "two ext cells per thread");
    const int e1 = tid, e2 = tid + kThreads;
    const bool has2 = e2 < G::EXT;
    uint2 gen[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
    if (tl.gtab >= 0) {
        const uint2 *gt = reinterpret_cast<const uint2 *>(a.gtab) + tl.gtab;
        gen[0] = gt[e1];
        if (has2) gen[1] = gt[e2];
    }
    // FP32: this lane's B operands of the MFMA phase (D^T, K = m in steps of
    // 4), loaded before the other set-up loads so that the MFMA phase waits
    // for them and the loads issued before it, not for the halo prefetch
    float bD[3] = {0.0f, 0.0f, 0.0f};
    if constexpr (MF) {
        if (ns > 1) {
            const int row = tid & 15, kq = (tid & 63) >> 4;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int m = 4 * s + kq;
                if (row < ns && m < ns) bD[s] = a.D[B.d_off + row * kNsPad + m];
            }
        }
    }
    // geometry of this thread's i-face and j-face (one of each per thread):
    // the loads are issued here, the derived quantities formed after the
    // tile's first barrier, so that every load of the tile set-up (table,
    // faces, halo, own cells) is in flight at once
    static_assert(G::NFI <= kThreads && G::NFJ <= kThreads, "one face per thread and pass");
    T rI[4] = {T(1), T(0), T(1), T(0)}, rJ[4] = {T(1), T(0), T(1), T(0)};
    bool hasI, hasJ;
    // moving grid: body-frame midpoints of the two faces relative to the
    // pivot (the face speed of snapshot n follows from them)
    const int64_t nnod = (int64_t)(ni + 1) * (nj + 1);
    const double *X = MV ? a.xy + 2 * B.node_off : nullptr;
    T mIx = T(0), mIy = T(0), mJx = T(0), mJy = T(0);
    {
        const int fi = tid % (TI + 1), fj = tid / (TI + 1);
        const int gi = tl.i0 + fi, gj = tl.j0 + fj;
        hasI = tid < G::NFI && gi <= ni && gj < nj;
        if (hasI) {
            const unsigned fg = (unsigned)(gj * (ni + 1) + gi);
            const int nf = (ni + 1) * nj;
            rI[0] = ldg(tu.SI, fg); rI[1] = ldg(tu.SI + nf, fg);
            rI[2] = ldg(tu.dI, fg); rI[3] = ldg(tu.dI + nf, fg);
            if constexpr (MV) {     // edge from node (gi, gj) to (gi, gj + 1)
                const unsigned k0 = (unsigned)(gj * (ni + 1) + gi), k1 = k0 + (unsigned)(ni + 1);
                mIx = (T)(0.5 * (ldg(X, k0) + ldg(X, k1)) - a.xp);
                mIy = (T)(0.5 * (ldg(X + nnod, k0) + ldg(X + nnod, k1)) - a.yp);
            }
        }
    }
    {
        const int fi = tid % TI, fj = tid / TI;
        const int gi = tl.i0 + fi, gj = tl.j0 + fj;
        hasJ = tid < G::NFJ && gi < ni && gj <= nj;
        if (hasJ) {
            const unsigned fg = (unsigned)(gj * ni + gi);
            const int nf = ni * (nj + 1);
            rJ[0] = ldg(tu.SJ, fg); rJ[1] = ldg(tu.SJ + nf, fg);
            rJ[2] = ldg(tu.dJ, fg); rJ[3] = ldg(tu.dJ + nf, fg);
            if constexpr (MV) {     // edge from node (gi, gj) to (gi + 1, gj)
                const unsigned k0 = (unsigned)(gj * (ni + 1) + gi), k1 = k0 + 1u;
                mJx = (T)(0.5 * (ldg(X, k0) + ldg(X, k1)) - a.xp);
                mJy = (T)(0.5 * (ldg(X + nnod, k0) + ldg(X + nnod, k1)) - a.yp);
            }
        }
    }
    // moving grid: the cell centre relative to the pivot (time step of the
    // first stage), and for each of this thread's ghost-extended cells that
    // is a moving no-slip wall image, the body-frame midpoint of its wall
    // face relative to the pivot
    T cxr = T(0), cyr = T(0);
    T wmx[2] = {T(0), T(0)}, wmy[2] = {T(0), T(0)};
    bool wimg[2] = {false, false};
    if constexpr (MV) {
        if constexpr (FIRST && MODE != 0) {
            const double *Cx = a.C + 2 * B.cell_off;
            cxr = (T)(ldg(Cx, cidx) - a.xp);
            cyr = (T)(ldg(Cx + plane, cidx) - a.yp);
        }
        if (tl.gtab >= 0) {
            const uint2 *wt = reinterpret_cast<const uint2 *>(a.wtab) + tl.gtab;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c && !has2) break;
                const uint2 w = wt[c ? e2 : e1];
                if (w.y != 0u) {
                    wimg[c] = true;
                    const double *x = a.xy + w.x, *y = x + w.y;
                    wmx[c] = (T)(0.5 * (x[0] + x[1]) - a.xp);
                    wmy[c] = (T)(0.5 * (y[0] + y[1]) - a.yp);
                }
            }
        }
    }

    // own-cell state of snapshot m, variable v (perturbation form)
    const double *q0b = a.q0 + B.q_off;
    auto load_own = [&](int m, int v) -> T {
        if (!valid) return T(0);
        if constexpr (FIRST)
            return (T)(ldg(q0b + (m * 4 + v) * plane, cidx) - a.ffq[4 * (B.snap_off + m) + v]);
        else
            return ldg(a.sin + B.q_off + (m * 4 + v) * plane, cidx);
    };
    // Later stages (FP32): the own-cell state of every snapshot is loaded now,
    // so that these loads are in flight together with the ghost-source
    // resolution and the first halo prefetch below (their waits overlap).
    constexpr bool EARLY = MF && !FIRST;
    T own[EARLY ? kMaxNs : 1][4];
    if constexpr (EARLY) {
#pragma unroll
        for (int m = 0; m < kMaxNs; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) own[m][v] = (m < ns && ns > 1) ? load_own(m, v) : T(0);
    }

    // geometry of the own cell: the area and, for the time step (formed by
    // the first stage of an iteration), the mean face normals.  Loaded by
    // every lane (cell 0 for the helper row and cells outside the block).
    T sxi = T(0), syi = T(0), sxj = T(0), syj = T(0);
    if constexpr (FIRST && MODE != 0) {
        const int nfi = (ni + 1) * nj, nfj = ni * (nj + 1);
        const unsigned fi0 = valid ? (unsigned)(j * (ni + 1) + i) : 0u;
        const T *SIx = a.SI + 2 * B.fi_off, *SIy = SIx + nfi;
        const T *SJx = a.SJ + 2 * B.fj_off, *SJy = SJx + nfj;
        sxi = T(0.5) * (ldg(SIx, fi0) + ldg(SIx + 1, fi0));
        syi = T(0.5) * (ldg(SIy, fi0) + ldg(SIy + 1, fi0));
        sxj = T(0.5) * (ldg(SJx, cidx) + ldg(SJx + ni, cidx));
        syj = T(0.5) * (ldg(SJy, cidx) + ldg(SJy + ni, cidx));
    }
    const T vraw = ldg(a.V + B.cell_off, cidx);
    const T vol = valid ? vraw : T(1);
    const double ivol = 1.0 / (double)vol;

    // Sources of this thread's two ghost-extended cells (tid and tid + 256),
    // the same for every snapshot.  In a tile away from the block sides
    // every ext cell is a cell of the block; a tile at a side reads them from
    // its halo source table, where the ghost rules were applied on the host
    // (an interior cell of some block, or the far field, with the parity of
    // wall mirrors).  Every snapshot's values are then loaded one snapshot
    // ahead into registers.  A source is a byte offset into the whole state
    // array (the state below 4 GiB, so that it fits 32 bits; BIG: a 64-bit
    // element offset) and its block's plane in the same unit; the four
    // variables of a snapshot are one plane apart, the next snapshot four.
    using LT = std::conditional_t<FIRST, double, T>;
    using OT = std::conditional_t<BIG, uint64_t, unsigned>;
    constexpr OT kUnit = BIG ? 1 : sizeof(LT);
    LT pf[2][4] = {};         // never loaded for far-field sources
    OT sbo[2] = {0u, 0u}, sbp[2] = {0u, 0u};
    int sff[2] = {1, 1}, smir[2] = {0, 0};       // far field: no load
    if (tl.gtab < 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int e = c ? e2 : e1;
            if (c && !has2) break;
            const int gi = tl.i0 + e % G::WE - 2, gj = tl.j0 + e / G::WE - 2;
            sff[c] = 0;
            sbo[c] = (OT)(B.q_off + gj * ni + gi) * kUnit;
            sbp[c] = (OT)plane * kUnit;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c && !has2) break;
            const uint2 en = gen[c];
            sff[c] = en.y == 0u;
            smir[c] = (int)(en.x >> 31);
            if constexpr (BIG) sbo[c] = a.gtab64[tl.gtab + (c ? e2 : e1)];
            else sbo[c] = (en.x & 0x7fffffffu) * kUnit;
            sbp[c] = (OT)en.y * kUnit;
        }
    }
    const LT *src0;
    if constexpr (FIRST) src0 = a.q0;
    else src0 = a.sin;
    // loads snapshot m's values and advances the offsets to snapshot m + 1
    auto prefetch = [&]() {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (!sff[c] && (c == 0 || has2)) {
                OT o = sbo[c];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (BIG) pf[c][v] = src0[o];
                    else pf[c][v] = ldgb(src0, o);
                    o += sbp[c];
                }
                sbo[c] = o;
            }
        }
    };
    prefetch();

    if (wtf) Tf[tid] = tfv;
    else if (wtd) Td[tid - 128] = tdv;

    // ---- A + B: HB source D (Q - Q_inf) of the tile ----------------------
    T dq[MF ? 1 : (NS > 0 ? NS : 1)][4];
    if constexpr (MF) {
        if (ns > 1) {
            if constexpr (EARLY) {
#pragma unroll
                for (int m = 0; m < kMaxNs; ++m)
                    if (m < ns)
#pragma unroll
                        for (int v = 0; v < 4; ++v) DQs[(m * 4 + v) * kDqS + tid] = own[m][v];
            } else {
#pragma unroll 3
                for (int m = 0; m < ns; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v) DQs[(m * 4 + v) * kDqS + tid] = load_own(m, v);
            }
            __syncthreads();
            // per var v and 16-cell group cb: the 16x16 block (cells x n) =
            // Q^T[cells x m] * D^T[m x n], K = m in steps of 4 (v_mfma 16x16x4).
            // Wave w takes groups w, w + 4, ..., kBatch at a time: the operands
            // of the batch are read from LDS first and their MFMA chains then
            // interleave, so that the wave waits for LDS once per batch
            // rather than before every MFMA.
            const int lane = tid & 63, wave = tid >> 6;
            const int row = lane & 15, kq = lane >> 4;
            const int KS = (ns + 3) / 4;            // <= 3
            constexpr int kGroups = 4 * (kThreads / 16);          // (v, cb) groups
            constexpr int kPerWave = kGroups / (kThreads / 64);
            constexpr int kBatch = 2;                              // groups per LDS wait
#pragma unroll 1
            for (int k = 0; k < kPerWave; k += kBatch) {
                float av[kBatch][3];
#pragma unroll
                for (int bq = 0; bq < kBatch; ++bq) {
                    const int grp = wave + (kThreads / 64) * (k + bq);
                    const int v = grp / (kThreads / 16), cb = grp % (kThreads / 16);
#pragma unroll
                    for (int s = 0; s < 3; ++s) {
                        const int m = 4 * s + kq;
                        const int mc = m < ns ? m : ns - 1;        // in range; zeroed below
                        const float x = DQs[(mc * 4 + v) * kDqS + cb * 16 + row];
                        av[bq][s] = m < ns ? x : 0.0f;
                    }
                }
                floatx4 acc[kBatch];
#pragma unroll
                for (int bq = 0; bq < kBatch; ++bq) acc[bq] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    if (s < KS) {
#pragma unroll
                        for (int bq = 0; bq < kBatch; ++bq)
                            acc[bq] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bq][s], bD[s], acc[bq], 0, 0, 0);
                    }
                }
                // lane holds (cell cb*16 + 4 kq + r, n = row); written in
                // place: only this wave reads or writes group (v, cb), and
                // every read feeds the MFMAs before the results exist
                if (row < ns) {
#pragma unroll
                    for (int bq = 0; bq < kBatch; ++bq) {
                        const int grp = wave + (kThreads / 64) * (k + bq);
                        const int v = grp / (kThreads / 16), cb = grp % (kThreads / 16);
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            DQs[(row * 4 + v) * kDqS + cb * 16 + 4 * kq + r] = acc[bq][r];
                    }
                }
            }
            // the first barrier of the snapshot loop orders these writes
            // before their reads
        }
    } else {
        T qp[NS][4];
#pragma unroll
        for (int m = 0; m < NS; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) qp[m][v] = load_own(m, v);
#pragma unroll
        for (int n = 0; n < NS; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T s = T(0);
#pragma unroll
                for (int m = 0; m < NS; ++m) s += a.D[B.d_off + n * kNsPad + m] * qp[m][v];
                dq[n][v] = s;
            }
    }

    // the table (and, without the MFMA phase, everything else) must be
    // visible before the snapshot loop
    if (!(MF && ns > 1)) __syncthreads();
    const FaceGeo<T> gI = face_geo<T>(rI[0], rI[1], rI[2], rI[3], a.mu, a.kappa);
    const FaceGeo<T> gJ = face_geo<T>(rJ[0], rJ[1], rJ[2], rJ[3], a.mu, a.kappa);
    // moving grid: the rigid velocity theta_dot k x R (x0 - p) + (0, h_dot)
    // at a face midpoint x0, dotted with the rotated normal R n, is
    // theta_dot (k x (x0 - p)) . n + h_dot (R n)_y: the first factor is the
    // same for every snapshot
    const T wI = MV ? mIx * gI.ny - mIy * gI.nx : T(0);
    const T wJ = MV ? mJx * gJ.ny - mJy * gJ.nx : T(0);

    // ---- C: snapshot loop -----------------------------------------------
    double nacc = 0.0;
    const int iw = tj * (TI + 1) + ti, js = tj * TI + ti;
    for (int n = 0; n < ns; ++n) {
        // base state of this snapshot for the update (loaded early)
        const int so = n * 4 * plane;     // snapshot offset (uniform)
        double b0[4] = {0.0, 0.0, 0.0, 0.0};
        // local time step: formed from the base state by the first stage,
        // which stores it; later stages load it (it is frozen over the stages)
        T* const dtb = a.dtau + B.q_off / 4 + n * plane;
        T dt = T(0);
        if constexpr (MODE != 0) {
            // unconditional (cidx = 0 for the helper row and cells outside
            // the block): a fixed count of loads lets the halo values of
            // this snapshot be consumed without waiting for these
#pragma unroll
            for (int v = 0; v < 4; ++v) b0[v] = ldg(q0b + so + v * plane, cidx);
            if constexpr (!FIRST) dt = ldg(dtb, cidx);
        }
        // moving grid: this snapshot's rotation and rates (uniform loads)
        T mc = T(1), ms = T(0), mthd = T(0), mhd = T(0);
        if constexpr (MV) {
            const double *mt = a.mot + kMotionW * (B.snap_off + n);
            mc = (T)mt[0];
            ms = (T)mt[1];
            mthd = (T)mt[2];
            mhd = (T)mt[4];
        }
        const T *fw = Tf + 8 * n;
        FS<T> f;
        f.u = fw[0];
        f.v = fw[1];
        f.p = fw[2];
        f.gg = g / gm1;
        f.h = f.gg * f.p + T(0.5) * (f.u * f.u + f.v * f.v);
        // C1: ghost-extended tile from the prefetch registers; then the next
        // snapshot's loads are issued
        {
            const double *fq = Td + 4 * n;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int e = c ? e2 : e1;
                if (c && !has2) break;
                T d[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (FIRST) d[v] = sff[c] ? T(0) : (T)(pf[c][v] - fq[v]);
                    else d[v] = pf[c][v];       // far-field sources keep their zero
                }
                T tp;
                W4<T> w = pert_prim_t<T>(d[0], d[1], d[2], d[3], f.u, f.v, gm1, g, tp);
                if (smir[c]) {                  // no-slip wall image: velocity reversed
                    w.u = -w.u - T(2) * f.u;
                    w.v = -w.v - T(2) * f.v;
                }
                if constexpr (MV) {
                    if (wimg[c]) {              // moving wall: u_g = 2 u_wall - u
                        const T rx = mc * wmx[c] - ms * wmy[c], ry = ms * wmx[c] + mc * wmy[c];
                        w.u += T(2) * (-mthd * ry);
                        w.v += T(2) * (mthd * rx + mhd);
                    }
                }
                P[e] = w.r;
                P[G::EXT + e] = w.u;
                P[2 * G::EXT + e] = w.v;
                P[3 * G::EXT + e] = w.p;
                P[4 * G::EXT + e] = tp;
            }
            if (n + 1 < ns) prefetch();
        }
        __syncthreads();
        // C2: node averages of (u', v', T')
        for (int k = tid; k < G::NOD; k += kThreads) {
            const int a0 = k % (TI + 1), b0 = k / (TI + 1);
            const int e00 = (b0 + 1) * G::WE + a0 + 1;
            const int e01 = e00 + G::WE;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T *pc = P + (c == 2 ? 4 : c + 1) * G::EXT;
                Nd[c * G::NOD + k] = T(0.25) * (pc[e00] + pc[e00 + 1] + pc[e01] + pc[e01 + 1]);
            }
        }
        // this snapshot's HB source into registers (the MFMA results of the
        // tile are ordered before these reads by the barrier above); its LDS
        // slot then receives the j-face fluxes
        T dqv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if constexpr (MF) dqv[v] = (ns > 1) ? DQs[(n * 4 + v) * kDqS + tid] : T(0);
            else dqv[v] = dq[0][v];
        }
        T *FJ = MF ? DQs + n * 4 * kDqS : FJ64;
        constexpr int fjs = MF ? kDqS : G::NFMAX;
        __syncthreads();
        // C3: i-face and j-face fluxes, each face once
        if constexpr (MV) {
            const FaceGeo<T> hI = rotate_geo(gI, mc, ms), hJ = rotate_geo(gJ, mc, ms);
            if (hasI) face_flux<T, TI, TJ, true, true>(a, tid, P, Nd, F, G::NFMAX, f, hI,
                                                       mthd * wI + mhd * hI.ny);
            if (hasJ) face_flux<T, TI, TJ, false, true>(a, tid, P, Nd, FJ, fjs, f, hJ,
                                                        mthd * wJ + mhd * hJ.ny);
        } else {
            if (hasI) face_flux<T, TI, TJ, true, false>(a, tid, P, Nd, F, G::NFMAX, f, gI, T(0));
            if (hasJ) face_flux<T, TI, TJ, false, false>(a, tid, P, Nd, FJ, fjs, f, gJ, T(0));
        }
        __syncthreads();
        // C4: cell residual and update
        if (valid) {
            T rs[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                rs[v] = F[v * G::NFMAX + iw + 1] - F[v * G::NFMAX + iw];
                rs[v] += (FJ[v * fjs + js + TI] - FJ[v * fjs + js]) + vol * (dqv[v] + fw[4 + v]);
            }
            if constexpr (MODE == 0) {
                double *ob = a.qout + B.q_off + so;
#pragma unroll
                for (int v = 0; v < 4; ++v) stg(ob + v * plane, cidx, (double)rs[v]);
            } else {
                const double *fq = Td + 4 * n;
                if constexpr (FIRST) {
                    const W4<T> wp = pert_prim<T>((T)(b0[0] - fq[0]), (T)(b0[1] - fq[1]),
                                                  (T)(b0[2] - fq[2]), (T)(b0[3] - fq[3]), f.u, f.v, gm1);
                    if constexpr (MV) {
                        // the snapshot's mean normals; velocity relative to
                        // the grid at the cell centre
                        const T rx = mc * cxr - ms * cyr, ry = ms * cxr + mc * cyr;
                        const W4<T> wf{T(1) + wp.r, f.u + wp.u + mthd * ry,
                                       f.v + wp.v - (mthd * rx + mhd), f.p + wp.p};
                        dt = local_dt<T>(wf, mc * sxi - ms * syi, ms * sxi + mc * syi,
                                         mc * sxj - ms * syj, ms * sxj + mc * syj, vol, g, a.mu_pr,
                                         a.cfl, (T)B.omega_nh);
                    } else {
                        const W4<T> wf{T(1) + wp.r, f.u + wp.u, f.v + wp.v, f.p + wp.p};
                        dt = local_dt<T>(wf, sxi, syi, sxj, syj, vol, g, a.mu_pr, a.cfl, (T)B.omega_nh);
                    }
                    stg(dtb, cidx, dt);
                }
                const double fac = a.alpha * (double)dt * ivol;
                double nq[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) nq[v] = b0[v] - fac * (double)rs[v];
                if constexpr (MODE == 1) {
                    T *sb = a.sout + B.q_off + so;
#pragma unroll
                    for (int v = 0; v < 4; ++v) stg(sb + v * plane, cidx, (T)(nq[v] - fq[v]));
                } else {
                    double *ob = a.qout + B.q_off + so;
#pragma unroll
                    for (int v = 0; v < 4; ++v) stg(ob + v * plane, cidx, nq[v]);
                }
                // density > 0 and pressure > 0 (rho E rho > |rho u|^2 / 2), finite residual
                const double pr = nq[3] * nq[0] - 0.5 * (nq[1] * nq[1] + nq[2] * nq[2]);
                if (!(nq[0] > 0.0) || !(pr > 0.0) || !isfinite((double)(rs[0] + rs[1] + rs[2] + rs[3])))
                    bad = 1;
            }
            const double rr = (double)rs[0] * ivol;
            nacc += rr * rr;
        }
        if constexpr (!MF) {
            // rotate the HB source so that dq[0] belongs to the next snapshot
#pragma unroll
            for (int m = 0; m + 1 < NS; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) dq[m][v] = dq[m + 1][v];
        }
    }
    if (a.norm) {
        // deterministic tile partial: wave reduction, then 4 waves in order
        for (int off = 32; off > 0; off >>= 1) nacc += __shfl_xor(nacc, off, 64);
        __shared__ double wsum[kThreads / 64];
        __syncthreads();
        if ((tid & 63) == 0) wsum[tid >> 6] = nacc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) s += wsum[w];
            a.partials[tile_id] = s;
        }
    }
}

template <class T, int TI, int TJ, bool FIRST, int MODE, bool MV, bool BIG>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MV) ? 3 : 1)))
k_fused(FusedArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its
    // own L2).  Renumber them so that the workgroups of one XCD take
    // consecutive tiles of the list at the same time: neighbouring tiles,
    // whose halos overlap, then share an L2.  The list is cut into rounds of
    // 8 chunks of C = a.xcd tiles; the k-th workgroup of XCD x takes tile
    // k % C of chunk x of round k / C, so that all XCDs move through the
    // list (sorted by snapshot count) together.  A permutation when the
    // grid is a multiple of 8 C, which the host ensures.
    const int G = gridDim.x;
    int v0 = blockIdx.x;
    if (a.xcd > 0 && G % (8 * a.xcd) == 0) {
        const int C = a.xcd, x = blockIdx.x % 8, k = blockIdx.x / 8;
        v0 = (k / C) * 8 * C + x * C + k % C;
    }
    int bad = 0;          // a cell of any of this workgroup's tiles went bad
    for (int t = v0; t < a.n_tiles; t += G) {
        const Tile tg = a.tiles[t];
        const Tile tl{uni(tg.blk), uni(tg.i0), uni(tg.j0), uni(tg.ns), uni(tg.gtab)};
        if constexpr (std::is_same<T, float>::value) {
            tile_body<T, TI, TJ, FIRST, MODE, 0, MV, BIG>(a, tl, t, smem, bad);
        } else {
            switch (tl.ns) {
                case 1: tile_body<T, TI, TJ, FIRST, MODE, 1, MV, BIG>(a, tl, t, smem, bad); break;
                case 3: tile_body<T, TI, TJ, FIRST, MODE, 3, MV, BIG>(a, tl, t, smem, bad); break;
                case 5: tile_body<T, TI, TJ, FIRST, MODE, 5, MV, BIG>(a, tl, t, smem, bad); break;
                case 7: tile_body<T, TI, TJ, FIRST, MODE, 7, MV, BIG>(a, tl, t, smem, bad); break;
                default: tile_body<T, TI, TJ, FIRST, MODE, 9, MV, BIG>(a, tl, t, smem, bad); break;
            }
        }
        __syncthreads();
    }
    // at most one atomic per wave and launch: a diverging state must not
    // turn into one atomic per cell on a single word
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(a.status, 1);
}

// FP32: the HB-source slots, one per snapshot (at least one: it also holds
// the j-face fluxes of the snapshot being computed)
template <class T, int TI, int TJ>
size_t dq_bytes(int ns_max) {
    static_assert(Geo<TI, TJ>::NFJ <= kDqS, "j-face fluxes fit a HB-source slot");
    return std::is_same<T, float>::value ? sizeof(float) * (size_t)std::max(ns_max, 1) * 4 * kDqS : 0;
}

template <class T, int TI, int TJ>
size_t smem_bytes(int ns_max) {
    // HB-source slots (FP32), scratch, the FP64 j-face area, then the
    // per-snapshot table (8 T + 4 doubles per snapshot)
    using G = Geo<TI, TJ>;
    const size_t fj = std::is_same<T, float>::value ? 0 : 4 * (size_t)G::NFMAX;
    return dq_bytes<T, TI, TJ>(ns_max) + sizeof(T) * ((size_t)G::SCRATCH + fj + 8 * kMaxNs) +
           sizeof(double) * 4 * kMaxNs;
}

inline int ns_max(const hb_grid *g) {
    int m = 1;
    for (const BlockDesc &B : g->blk) m = std::max(m, B.ns);
    return m;
}

// tiles per XCD chunk of a one-workgroup-per-tile grid with the XCD renumbering
constexpr int kXcdChunk = 32;

template <class T, int TI, int TJ, bool FIRST, int MODE, bool MV, bool BIG>
int launch_t(hb_grid *g, const FusedArgs<T> &a, hipStream_t s) {
    const size_t sm = smem_bytes<T, TI, TJ>(ns_max(g));
    FusedArgs<T> b = a;
    b.dq_bytes = (int)dq_bytes<T, TI, TJ>(ns_max(g));
    auto kern = k_fused<T, TI, TJ, FIRST, MODE, MV, BIG>;
    // persistent grid: as many workgroups as can be resident at once
    static int cached_occ[2][2] = {{0, 0}, {0, 0}};
    static size_t cached_sm[2][2] = {{0, 0}, {0, 0}};
    int &occ = cached_occ[FIRST][MODE == 2];
    if (!occ || cached_sm[FIRST][MODE == 2] != sm) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kThreads, sm) != hipSuccess || nb < 1)
            nb = 1;
        occ = nb;
        cached_sm[FIRST][MODE == 2] = sm;
    }
    // wg_per_cu < 0: one workgroup per tile (the dispatcher starts a tile
    // whenever a workgroup slot frees), the grid rounded up to a multiple of
    // 8 when the XCD renumbering is on (the extra workgroups find no tile);
    // else a persistent grid
    const int per_cu = g->tune_wg_per_cu > 0 ? std::min(g->tune_wg_per_cu, occ) : occ;
    int grid = g->tune_wg_per_cu < 0 ? std::max(1, g->n_tiles)
                                     : std::max(1, std::min(g->n_tiles, g->n_cu * per_cu));
    b.xcd = 0;
    if (g->tune_xcd) {
        if (g->tune_wg_per_cu < 0) {
            b.xcd = kXcdChunk;
            grid = (grid + 8 * kXcdChunk - 1) / (8 * kXcdChunk) * (8 * kXcdChunk);
        } else if (grid % 8 == 0) {
            b.xcd = grid / 8;        // persistent grid: one chunk per XCD and round
        }
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), sm, s, b);
    return check_hip(hipGetLastError(), "fused launch");
}

template <class T, bool FIRST, int MODE, bool MV, bool BIG>
int launch_shape(hb_grid *g, const FusedArgs<T> &a, hipStream_t s) {
    if (g->tile_ti == 32) return launch_t<T, 32, 8, FIRST, MODE, MV, BIG>(g, a, s);
    return launch_t<T, 16, 16, FIRST, MODE, MV, BIG>(g, a, s);
}

// One stage launch of the variant (MV, BIG): first = the iteration's first
// stage, mode 0 = residual, 1 = intermediate stage, 2 = last stage.
// Instantiated once per variant in hb_fused_k*.hip.
template <class T, bool MV, bool BIG>
int launch_stage(hb_grid *g, const FusedArgs<T> &a, bool first, int mode, hipStream_t s) {
    if (first) {
        if (mode == 0) return launch_shape<T, true, 0, MV, BIG>(g, a, s);
        if (mode == 1) return launch_shape<T, true, 1, MV, BIG>(g, a, s);
        return fail(HB_ERR_UNSUPPORTED, "one-stage schemes are not supported by the fused path");
    }
    if (mode == 1) return launch_shape<T, false, 1, MV, BIG>(g, a, s);
    return launch_shape<T, false, 2, MV, BIG>(g, a, s);
}

}  // namespace fk
}  // namespace hb

