"""Seeded synthetic inputs: grids, flow/solver settings and initial states.

This module is shared by the HIP path's callers (bench, tests) and by the
tests that feed the FP64 CPU oracle.  It holds none of the method's
arithmetic: no metrics, fluxes, HB operator, time step or update.  It only
produces node coordinates, boundary-condition tags, scalar settings and the
seeded initial state, all as NumPy FP64 arrays, and imports nothing but NumPy.

The paper's own grids (a 512-block wing and a 2048-block blade section,
§Experimental Setup) are not available; the workloads below are synthetic
stand-ins with the structure the paper describes: structured multi-block
grids, 2*nharms+1 snapshots per block, npde = 4 conserved variables per
snapshot (§MPI Optimisations, halo pseudo code).

Conventions
-----------
* Node coordinates of a block: ``xy[2][nj+1][ni+1]`` (x then y), i fastest.
  The grid is right-handed: i runs along the body (clockwise), j outward.
* Boundary tags per side (imin, imax, jmin, jmax): WALL, FARFIELD, PERIODIC,
  CUT, WAKECUT (C-grid wake on jmin; cells i < wake_ncells and
  i >= ni - wake_ncells face each other across the cut, the rest is wall),
  CUT_WALL and CUT_FARFIELD (partly glued: the cells that cut segments cover
  are glued, the rest is wall or far field).
* Snapshot n of N_s = 2*N_H+1 sits at phase 2*pi*n/N_s of the period.
* State layout of one block: ``q[N_s][4][nj][ni]`` FP64, conserved
  (rho, rho*u, rho*v, rho*E); blocks are concatenated in order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

WALL, FARFIELD, PERIODIC, CUT, WAKECUT, CUT_WALL, CUT_FARFIELD = 1, 2, 3, 4, 5, 6, 7


# --------------------------------------------------------------------------
# Settings
# --------------------------------------------------------------------------
@dataclass
class Flow:
    """Free-stream and forcing settings (non-dimensional: rho_inf = 1,
    c_inf = 1, p_inf = 1/gamma, |V_inf| = mach, reference length 1).

    The incidence is alpha(t) = alpha0 + alpha_amp*sin(omega*t) with
    omega = 2*k_red*mach/l_ref (reduced frequency on the half chord).
    Angles are radians.  (x_mom, y_mom) is the moment reference point.
    """
    mach: float
    reynolds: float
    prandtl: float = 0.72
    gamma: float = 1.4
    alpha0: float = 0.0
    alpha_amp: float = 0.0
    k_red: float = 0.0
    l_ref: float = 1.0
    x_mom: float = 0.0
    y_mom: float = 0.0

    @property
    def omega(self) -> float:
        return 2.0 * self.k_red * self.mach / self.l_ref


@dataclass
class Solver:
    """Pseudo-time settings: four-stage low-storage Runge-Kutta with local
    time stepping.  precision: 0 = FP64, 1 = FP32 bulk (flux/source in FP32,
    state/update/norms/forces in FP64).

    CFL: with dtau = CFL V / (Lambda_I + Lambda_J + ...), the upwind
    operator's odd-even mode has the eigenvalue -2 CFL dtau-scaled, and the
    four-stage scheme with these coefficients (the classical RK4 polynomial
    for linear problems) is stable on the negative real axis down to
    about -2.785, so CFL <= 1.39.  The default is 1.0; the cylinder workload
    states 1.5 and keeps it."""
    cfl: float = 1.0
    n_stages: int = 4
    rk_alpha: Tuple[float, ...] = (0.25, 1.0 / 3.0, 0.5, 1.0)
    precision: int = 0
    entropy_delta: float = 0.1
    limiter_eps: float = 1e-12
    batched: int = 1
    graph_iters: int = 1


@dataclass
class Block:
    ni: int
    nj: int
    n_harm: int
    xy: np.ndarray                       # [2][nj+1][ni+1] float64
    bc: Tuple[int, int, int, int]        # imin, imax, jmin, jmax
    wake_ncells: int = 0
    body_id: int = 0

    @property
    def ns(self) -> int:
        return 2 * self.n_harm + 1

    @property
    def n_state(self) -> int:
        return self.ns * 4 * self.nj * self.ni


@dataclass
class Problem:
    name: str
    blocks: List[Block]
    flow: Flow
    solver: Solver
    n_iter: int
    seed: int
    design: Optional[dict] = None        # Hicks-Henne data (cfg4)
    notes: str = ""
    cuts: List[Tuple[int, int, int, int]] = field(default_factory=list)

    @property
    def cell_snapshots(self) -> int:
        return sum(b.ns * b.ni * b.nj for b in self.blocks)

    @property
    def n_state(self) -> int:
        return sum(b.n_state for b in self.blocks)

    @property
    def nbody(self) -> int:
        return max(b.body_id for b in self.blocks) + 1


# --------------------------------------------------------------------------
# Grid generators
# --------------------------------------------------------------------------
def stretch(eta: np.ndarray, ratio: float = 1.1, n_ref: int = 32) -> np.ndarray:
    """Wall-normal distribution s(eta) = (r^(n_ref*eta) - 1)/(r^n_ref - 1);
    with n_ref cells this is a geometric progression of ratio r."""
    return (ratio ** (n_ref * eta) - 1.0) / (ratio ** n_ref - 1.0)


def o_grid(ni: int, nj: int, r_in: float = 1.0, r_out: float = 20.0) -> np.ndarray:
    """O-grid around a circle of radius r_in: theta_i = -2*pi*i/ni (clockwise,
    so that j runs outward and the grid is right-handed), r_j = r_in +
    (r_out - r_in)*s(j/nj).  Node ni repeats node 0 bit for bit."""
    i = np.arange(ni + 1)
    theta = -2.0 * np.pi * (i % ni) / ni
    r = r_in + (r_out - r_in) * stretch(np.arange(nj + 1) / nj)
    x = r[:, None] * np.cos(theta)[None, :]
    y = r[:, None] * np.sin(theta)[None, :]
    return np.stack([x, y]).astype(np.float64)


def naca00_thickness(x: np.ndarray, t: float = 0.12) -> np.ndarray:
    """Symmetric NACA 4-digit half thickness, closed trailing edge."""
    xc = np.clip(x, 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(xc) - 0.1260 * xc - 0.3516 * xc ** 2
                      + 0.2843 * xc ** 3 - 0.1036 * xc ** 4)


def c_grid_inner(ni: int, t: float = 0.12, wake_len: float = 10.0,
                 wake_beta: float = 7.0):
    """Inner (j = 0) curve of the C-grid: lower wake (x from 1+wake_len to 1),
    lower surface (TE -> LE, cosine clustered), upper surface (LE -> TE),
    upper wake.  Returns x, y, and the surface flag per node."""
    assert ni % 4 == 0 and ni >= 8
    nw = ni // 4
    ns = ni // 4
    x = np.zeros(ni + 1)
    y = np.zeros(ni + 1)
    g = lambda s: (np.exp(wake_beta * s) - 1.0) / (np.exp(wake_beta) - 1.0)
    k = np.arange(nw + 1)
    x[:nw + 1] = 1.0 + wake_len * g((nw - k) / nw)
    k = np.arange(ns + 1)
    xl = 0.5 * (1.0 + np.cos(np.pi * k / ns))
    x[nw:nw + ns + 1] = xl
    y[nw:nw + ns + 1] = -naca00_thickness(xl, t)
    xu = 0.5 * (1.0 - np.cos(np.pi * k / ns))
    x[nw + ns:nw + 2 * ns + 1] = xu
    y[nw + ns:nw + 2 * ns + 1] = naca00_thickness(xu, t)
    k = np.arange(nw + 1)
    x[nw + 2 * ns:] = 1.0 + wake_len * g(k / nw)
    # exact closure at TE and LE
    x[nw] = x[nw + 2 * ns] = 1.0
    y[nw] = y[nw + 2 * ns] = 0.0
    y[nw + ns] = 0.0
    x[nw + ns] = 0.0
    surface = np.zeros(ni + 1, dtype=bool)
    surface[nw:nw + 2 * ns + 1] = True
    return x, y, surface


def c_grid_outer(ni: int, r_out: float = 10.0):
    """Outer C boundary: y = -r_out under the lower wake, a half circle of
    radius r_out centred on the trailing edge (1, 0) around the profile,
    y = +r_out over the upper wake."""
    xi, _, _ = c_grid_inner(ni)
    nw = ni // 4
    ns = ni // 4
    xo = np.zeros(ni + 1)
    yo = np.zeros(ni + 1)
    xo[:nw + 1] = xi[:nw + 1]
    yo[:nw + 1] = -r_out
    k = np.arange(2 * ns + 1)
    phi = -0.5 * np.pi - np.pi * k / (2 * ns)
    xo[nw:nw + 2 * ns + 1] = 1.0 + r_out * np.cos(phi)
    yo[nw:nw + 2 * ns + 1] = r_out * np.sin(phi)
    xo[nw + 2 * ns:] = xi[nw + 2 * ns:]
    yo[nw + 2 * ns:] = r_out
    xo[nw] = xo[nw + 2 * ns] = 1.0
    return xo, yo


def c_grid(ni: int, nj: int, t: float = 0.12, dy_surface: Optional[np.ndarray] = None
           ) -> np.ndarray:
    """C-grid around a symmetric NACA-00xx profile (chord 1, LE at origin).
    Nodes lie on straight lines from the inner curve to the outer C, with
    the wall-normal distribution s(eta).  dy_surface (optional, [ni+1])
    displaces the inner curve in y and decays as (1 - s(eta)) outward."""
    xi, yi, _ = c_grid_inner(ni, t)
    xo, yo = c_grid_outer(ni)
    s = stretch(np.arange(nj + 1) / nj)
    x = xi[None, :] + s[:, None] * (xo - xi)[None, :]
    y = yi[None, :] + s[:, None] * (yo - yi)[None, :]
    if dy_surface is not None:
        y = y + dy_surface[None, :] * (1.0 - s)[:, None]
    return np.stack([x, y]).astype(np.float64)


# --------------------------------------------------------------------------
# Hicks-Henne-style design variables (adjoint workload)
# --------------------------------------------------------------------------
def hicks_henne_basis(ni: int, n_per_side: int = 32) -> np.ndarray:
    """Bump functions b_k(x) = sin^3(pi * x^(ln 0.5 / ln h_k)), h_k = (k+1)/(n+1),
    evaluated at the inner-curve nodes: rows 0..n-1 act on the upper surface,
    rows n..2n-1 on the lower surface.  Returns B[2n][ni+1] (dy per unit beta).
    LE and TE nodes have b = 0, wake nodes are not displaced."""
    xi, _, surface = c_grid_inner(ni)
    nw = ni // 4
    ns = ni // 4
    upper = np.zeros(ni + 1, dtype=bool)
    upper[nw + ns:nw + 2 * ns + 1] = True
    lower = np.zeros(ni + 1, dtype=bool)
    lower[nw:nw + ns + 1] = True
    B = np.zeros((2 * n_per_side, ni + 1))
    for k in range(n_per_side):
        h = (k + 1.0) / (n_per_side + 1.0)
        e = math.log(0.5) / math.log(h)
        bx = np.sin(np.pi * np.clip(xi, 0.0, 1.0) ** e) ** 3
        B[k] = np.where(upper, bx, 0.0)
        B[n_per_side + k] = np.where(lower, bx, 0.0)
    B[:, nw] = B[:, nw + ns] = B[:, nw + 2 * ns] = 0.0
    return B


def hicks_henne_grid(ni: int, nj: int, beta: np.ndarray):
    """Deformed C-grid and its exact (linear) Jacobian dXY/dbeta.
    Returns xy [2][nj+1][ni+1] and dxy [nbeta][2][nj+1][ni+1]."""
    B = hicks_henne_basis(ni, len(beta) // 2)
    dy_s = beta @ B
    xy = c_grid(ni, nj, dy_surface=dy_s)
    s = stretch(np.arange(nj + 1) / nj)
    dxy = np.zeros((len(beta), 2, nj + 1, ni + 1))
    dxy[:, 1] = B[:, None, :] * (1.0 - s)[None, :, None]
    return xy, dxy


# --------------------------------------------------------------------------
# Initial state
# --------------------------------------------------------------------------
def initial_state(problem: Problem, seed: Optional[int] = None,
                  amplitude: float = 1e-3) -> np.ndarray:
    """Free stream at the snapshot's incidence plus a seeded Gaussian
    perturbation of the primitives (rho, u, v, p) of relative amplitude
    `amplitude` (scales rho_inf, |V_inf|, |V_inf|, p_inf).  Draws i.i.d.
    N(0,1) with NumPy PCG64 default_rng(seed), in public layout order
    block, n, v, j, i.  Returns the concatenated conserved state, FP64."""
    f = problem.flow
    rng = np.random.default_rng(problem.seed if seed is None else seed)
    g = f.gamma
    out = []
    for b in problem.blocks:
        ns = b.ns
        xi = rng.standard_normal((ns, 4, b.nj, b.ni))
        n = np.arange(ns)
        alpha = f.alpha0 + f.alpha_amp * np.sin(2.0 * np.pi * n / ns)
        rho = 1.0 + amplitude * xi[:, 0]
        u = (f.mach * np.cos(alpha))[:, None, None] + amplitude * f.mach * xi[:, 1]
        v = (f.mach * np.sin(alpha))[:, None, None] + amplitude * f.mach * xi[:, 2]
        p = 1.0 / g + amplitude * (1.0 / g) * xi[:, 3]
        q = np.stack([rho, rho * u, rho * v, p / (g - 1.0) + 0.5 * rho * (u * u + v * v)], axis=1)
        out.append(q.reshape(-1))
    return np.concatenate(out).astype(np.float64)


def block_offsets(problem: Problem) -> List[int]:
    off, o = [], 0
    for b in problem.blocks:
        off.append(o)
        o += b.n_state
    return off


def split_state(problem: Problem, q: np.ndarray) -> List[np.ndarray]:
    """View the concatenated state as per-block [N_s][4][nj][ni] arrays."""
    res = []
    for b, o in zip(problem.blocks, block_offsets(problem)):
        res.append(q[o:o + b.n_state].reshape(b.ns, 4, b.nj, b.ni))
    return res


def split_problem(problem: Problem, parts_i: int, parts_j: int):
    """Cut every block into parts_i x parts_j pieces glued by cuts (sides
    0..3 = imin, imax, jmin, jmax; a cut is (block_a, side_a, block_b,
    side_b), imax of a to imin of b or jmax of a to jmin of b).  A periodic
    side of a block that is cut along that direction becomes a cut between
    its first and last pieces.  Pieces are numbered block by block, j-piece
    major.  Returns (problem, perm) with state_split = state[perm].  A C-grid
    (wake-cut jmin) can only be cut along j."""
    blocks, cuts, perm = [], [], []
    off = 0
    for b in problem.blocks:
        if parts_i > 1 and b.bc[2] == WAKECUT:
            raise ValueError("a wake-cut block can only be split along j")
        ib = [round(k * b.ni / parts_i) for k in range(parts_i + 1)]
        jb = [round(k * b.nj / parts_j) for k in range(parts_j + 1)]
        base = len(blocks)
        idx = lambda pi, pj: base + pj * parts_i + pi
        for pj in range(parts_j):
            for pi in range(parts_i):
                i0, i1, j0, j1 = ib[pi], ib[pi + 1], jb[pj], jb[pj + 1]
                bc = list(b.bc)
                if parts_i > 1:
                    if pi > 0 or b.bc[0] == PERIODIC:
                        bc[0] = CUT
                    if pi < parts_i - 1 or b.bc[1] == PERIODIC:
                        bc[1] = CUT
                if parts_j > 1:
                    if pj > 0 or b.bc[2] == PERIODIC:
                        bc[2] = CUT
                    if pj < parts_j - 1 or b.bc[3] == PERIODIC:
                        bc[3] = CUT
                wake = b.wake_ncells if bc[2] == WAKECUT else 0
                xy = np.ascontiguousarray(b.xy[:, j0:j1 + 1, i0:i1 + 1])
                blocks.append(Block(i1 - i0, j1 - j0, b.n_harm, xy, tuple(bc), wake, b.body_id))
                n, v, j, i = np.meshgrid(np.arange(b.ns), np.arange(4), np.arange(j0, j1),
                                         np.arange(i0, i1), indexing="ij")
                perm.append((off + ((n * 4 + v) * b.nj + j) * b.ni + i).reshape(-1))
                if pi + 1 < parts_i:
                    cuts.append((idx(pi, pj), 1, idx(pi + 1, pj), 0))
                elif parts_i > 1 and b.bc[1] == PERIODIC:
                    cuts.append((idx(pi, pj), 1, idx(0, pj), 0))
                if pj + 1 < parts_j:
                    cuts.append((idx(pi, pj), 3, idx(pi, pj + 1), 2))
                elif parts_j > 1 and b.bc[3] == PERIODIC:
                    cuts.append((idx(pi, 0), 2, idx(pi, pj), 3))
        off += b.n_state
    out = Problem(problem.name + "_split%dx%d" % (parts_i, parts_j), blocks, problem.flow,
                  problem.solver, problem.n_iter, problem.seed, problem.design, problem.notes,
                  cuts)
    return out, np.concatenate(perm)


def _cell_perm(off: int, ns: int, nj: int, ni: int, j0: int, j1: int, i0: int, i1: int):
    """Public-layout indices of the cells [j0, j1) x [i0, i1) of a block at
    state offset off, in the layout of that sub-block."""
    n, v, j, i = np.meshgrid(np.arange(ns), np.arange(4), np.arange(j0, j1), np.arange(i0, i1),
                             indexing="ij")
    return (off + ((n * 4 + v) * nj + j) * ni + i).reshape(-1)


def split_c_grid(problem: Problem):
    """A one-block C-grid problem (wake-cut jmin) cut into three blocks
    along i: the lower wake, the part around the profile, the upper wake,
    glued by aligned cuts, and the wake cut as a reversed cut between the
    jmin sides of the two wake blocks (cut format of split_problem plus
    8-entry cuts (blk_a, side_a, start_a, blk_b, side_b, start_b, len,
    reversed)).  Returns (problem, perm) with state_split = state[perm]."""
    assert len(problem.blocks) == 1
    b = problem.blocks[0]
    assert b.bc[2] == WAKECUT and b.wake_ncells > 0
    w, ni, nj = b.wake_ncells, b.ni, b.nj
    parts = [(0, w, (b.bc[0], CUT, CUT, b.bc[3])), (w, ni - w, (CUT, CUT, WALL, b.bc[3])),
             (ni - w, ni, (CUT, b.bc[1], CUT, b.bc[3]))]
    blocks, perm = [], []
    for i0, i1, bc in parts:
        xy = np.ascontiguousarray(b.xy[:, :, i0:i1 + 1])
        blocks.append(Block(i1 - i0, nj, b.n_harm, xy, bc, 0, b.body_id))
        perm.append(_cell_perm(0, b.ns, nj, ni, 0, nj, i0, i1))
    cuts = [(0, 1, 1, 0), (1, 1, 2, 0), (0, 2, 0, 2, 2, 0, w, 1)]
    out = Problem(problem.name + "_c3", blocks, problem.flow, problem.solver, problem.n_iter,
                  problem.seed, problem.design, problem.notes, cuts)
    return out, np.concatenate(perm)


def c_grid_pieces(b: Block, ib: Sequence[int], jb: Sequence[int]):
    """A C-grid block (wake-cut jmin) cut at i positions ib and j positions
    jb (both including 0 and the size) into glued pieces, numbered j-layer
    major: (blocks, cuts, perm).  Neighbouring pieces are glued along whole
    sides; on the bottom layer the wake cells of a piece are glued (reversed)
    to the pieces holding their partners i <-> ni - 1 - i, so that a piece
    holding wake and profile cells has a partly glued jmin (CUT_WALL), one
    holding wake cells only a CUT jmin and one holding profile cells only a
    WALL jmin."""
    assert b.bc[2] == WAKECUT and b.wake_ncells > 0
    ni, nj, w = b.ni, b.nj, b.wake_ncells
    npi, npj = len(ib) - 1, len(jb) - 1
    idx = lambda pi, pj: pj * npi + pi
    blocks, cuts, perm = [], [], []
    for pj in range(npj):
        for pi in range(npi):
            i0, i1, j0, j1 = ib[pi], ib[pi + 1], jb[pj], jb[pj + 1]
            bc = [b.bc[0] if pi == 0 else CUT, b.bc[1] if pi == npi - 1 else CUT,
                  CUT, b.bc[3] if pj == npj - 1 else CUT]
            if pj == 0:
                nwake = sum(1 for i in range(i0, i1) if i < w or i >= ni - w)
                bc[2] = WALL if nwake == 0 else (CUT if nwake == i1 - i0 else CUT_WALL)
            xy = np.ascontiguousarray(b.xy[:, j0:j1 + 1, i0:i1 + 1])
            blocks.append(Block(i1 - i0, j1 - j0, b.n_harm, xy, tuple(bc), 0, b.body_id))
            perm.append(_cell_perm(0, b.ns, nj, ni, j0, j1, i0, i1))
            if pi + 1 < npi:
                cuts.append((idx(pi, pj), 1, idx(pi + 1, pj), 0))
            if pj + 1 < npj:
                cuts.append((idx(pi, pj), 3, idx(pi, pj + 1), 2))
    # wake: lower-wake cells [lo, hi) of piece p face cells [ni - hi, ni - lo) of piece q
    for p in range(npi):
        for q in range(npi):
            lo = max(ib[p], ni - ib[q + 1], 0)
            hi = min(ib[p + 1], ni - ib[q], w)
            if lo < hi:
                cuts.append((p, 2, lo - ib[p], q, 2, ni - hi - ib[q], hi - lo, 1))
    return blocks, cuts, np.concatenate(perm)


def split_c_grid_at(problem: Problem, ib: Sequence[int], jb: Sequence[int] = ()):
    """A one-block C-grid problem cut by c_grid_pieces at i positions ib and
    j positions jb (interior positions only).  Returns (problem, perm) with
    state_split = state[perm]."""
    assert len(problem.blocks) == 1
    b = problem.blocks[0]
    blocks, cuts, perm = c_grid_pieces(b, [0] + list(ib) + [b.ni], [0] + list(jb) + [b.nj])
    out = Problem(problem.name + "_cpieces", blocks, problem.flow, problem.solver, problem.n_iter,
                  problem.seed, problem.design, problem.notes, cuts)
    return out, perm


def c_grid_l(n_harm: int, scale: int = 1, body_id: int = 0):
    """Four uneven blocks of one C-grid of (448 x 160) / scale cells: the
    bottom layer (64 / scale rows) in three blocks of 256, 128 and 64
    columns (the lower wake and lower surface; the upper surface and the
    start of the upper wake; the rest of the upper wake), and one block of
    192 x 96 over the last two.  The wake is glued across the jmin sides of
    the bottom blocks (c_grid_pieces); the sides that face the part of the
    C-grid left out (the top of the first block, the imin side of the upper
    block) and the outer boundary are far field.  Returns (blocks, cuts)."""
    assert scale in (1, 2, 4, 8)
    ni, nj, h = 448 // scale, 160 // scale, 64 // scale
    big = Block(ni, nj, n_harm, c_grid(ni, nj), (FARFIELD, FARFIELD, WAKECUT, FARFIELD),
                ni // 4, body_id)
    ib = [0, 256 // scale, 384 // scale, ni]
    bottom, cuts, _ = c_grid_pieces(Block(ni, h, n_harm, np.ascontiguousarray(big.xy[:, :h + 1, :]),
                                          big.bc, big.wake_ncells, body_id), ib, [0, h])
    A, B, D = bottom
    bottom[0] = Block(A.ni, A.nj, n_harm, A.xy, (A.bc[0], A.bc[1], A.bc[2], FARFIELD), 0, body_id)
    bottom[1] = Block(B.ni, B.nj, n_harm, B.xy, (B.bc[0], B.bc[1], B.bc[2], CUT), 0, body_id)
    bottom[2] = Block(D.ni, D.nj, n_harm, D.xy, (D.bc[0], D.bc[1], D.bc[2], CUT), 0, body_id)
    top = Block(ni - ib[1], nj - h, n_harm, np.ascontiguousarray(big.xy[:, h:, ib[1]:]),
                (FARFIELD, FARFIELD, CUT, FARFIELD), 0, body_id)
    nb = ib[2] - ib[1]
    cuts = cuts + [(1, 3, 0, 3, 2, 0, nb, 0), (2, 3, 0, 3, 2, nb, ni - ib[2], 0)]
    return bottom + [top], cuts


def rotate_block(problem: Problem, k: int):
    """Block k re-indexed by a quarter turn of its index space (orientation
    kept): node (I, J) becomes (J, ni - I), cell (i, j) becomes
    (j, ni - 1 - i), so its imin, imax, jmin, jmax sides become jmax, jmin,
    imin, imax; its cuts follow (positions along its old j sides run the
    other way).  Returns (problem, perm) with state_rotated = state[perm]."""
    b = problem.blocks[k]
    assert b.bc[2] != WAKECUT
    ni, nj = b.ni, b.nj
    xy = np.ascontiguousarray(np.stack([b.xy[c].T[::-1, :] for c in range(2)]))
    bc = (b.bc[2], b.bc[3], b.bc[1], b.bc[0])
    blocks = list(problem.blocks)
    blocks[k] = Block(nj, ni, b.n_harm, xy, bc, 0, b.body_id)
    new_side = {0: 3, 1: 2, 2: 0, 3: 1}
    cuts = []
    for c in problem.cuts:
        if len(c) == 4:
            a, sa, bb, sb = c
            la = problem.blocks[a].nj if sa < 2 else problem.blocks[a].ni
            c = (a, sa, 0, bb, sb, 0, la, 0)
        a, sa, st_a, bb, sb, st_b, ln, rev = c
        if a == k:
            if sa >= 2:
                st_a, rev = ni - st_a - ln, 1 - rev
            sa = new_side[sa]
        if bb == k:
            if sb >= 2:
                st_b, rev = ni - st_b - ln, 1 - rev
            sb = new_side[sb]
        cuts.append((a, sa, st_a, bb, sb, st_b, ln, rev))
    offs = block_offsets(problem)
    perm = []
    for m, blk in enumerate(problem.blocks):
        idx = np.arange(offs[m], offs[m] + blk.n_state)
        if m == k:
            idx = idx.reshape(b.ns, 4, nj, ni)
            # new cell (i', j') = old (ni - 1 - j', i'): [n][v][j'][i']
            idx = np.ascontiguousarray(np.transpose(idx, (0, 1, 3, 2))[:, :, ::-1, :]).reshape(-1)
        perm.append(idx)
    out = Problem(problem.name + "_rot%d" % k, blocks, problem.flow, problem.solver,
                  problem.n_iter, problem.seed, problem.design, problem.notes, cuts)
    return out, np.concatenate(perm)


def split_partial(problem: Problem):
    """A one-block O-grid problem (i-periodic) cut into three blocks: the
    left half of i split in j into an inner and an outer block, and the
    right half whole, so that each i side of the right half is glued to two
    blocks by two segments.  Returns (problem, perm)."""
    assert len(problem.blocks) == 1
    b = problem.blocks[0]
    assert b.bc[0] == PERIODIC and b.bc[1] == PERIODIC
    ni, nj = b.ni, b.nj
    ih, jh = ni // 2, nj // 2
    parts = [(0, ih, 0, jh, (CUT, CUT, b.bc[2], CUT)), (0, ih, jh, nj, (CUT, CUT, CUT, b.bc[3])),
             (ih, ni, 0, nj, (CUT, CUT, b.bc[2], b.bc[3]))]
    blocks, perm = [], []
    for i0, i1, j0, j1, bc in parts:
        xy = np.ascontiguousarray(b.xy[:, j0:j1 + 1, i0:i1 + 1])
        blocks.append(Block(i1 - i0, j1 - j0, b.n_harm, xy, bc, 0, b.body_id))
        perm.append(_cell_perm(0, b.ns, nj, ni, j0, j1, i0, i1))
    cuts = [(0, 3, 1, 2),
            (0, 1, 0, 2, 0, 0, jh, 0), (1, 1, 0, 2, 0, jh, nj - jh, 0),
            (2, 1, 0, 0, 0, 0, jh, 0), (2, 1, jh, 1, 0, 0, nj - jh, 0)]
    out = Problem(problem.name + "_partial", blocks, problem.flow, problem.solver,
                  problem.n_iter, problem.seed, problem.design, problem.notes, cuts)
    return out, np.concatenate(perm)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
DEG = math.pi / 180.0


def o_block(ni, nj, n_harm, body_id=0) -> Block:
    return Block(ni, nj, n_harm, o_grid(ni, nj), (PERIODIC, PERIODIC, WALL, FARFIELD),
                 0, body_id)


def c_block(ni, nj, n_harm, body_id=0, xy=None) -> Block:
    return Block(ni, nj, n_harm, c_grid(ni, nj) if xy is None else xy,
                 (FARFIELD, FARFIELD, WAKECUT, FARFIELD), ni // 4, body_id)


def flow_cylinder() -> Flow:
    """Mach 0.3, Re 1000, incidence 2 deg amplitude, reduced frequency 0.1."""
    return Flow(mach=0.3, reynolds=1000.0, alpha_amp=2.0 * DEG, k_red=0.1)


def flow_airfoil() -> Flow:
    """Mach 0.5, Re 5000, pitching amplitude 1 deg, reduced frequency 0.2,
    moments about the quarter chord."""
    return Flow(mach=0.5, reynolds=5000.0, alpha_amp=1.0 * DEG, k_red=0.2, x_mom=0.25)


def cfg5_draw(seed: int = 7654, n_blocks: int = 32, target: float = 8e6):
    """Uneven block sizes and harmonic counts: ni ~ U[64,512], nj ~ U[32,128],
    N_H ~ U{1..4}; sizes rescaled by a common factor until the total is about
    `target` cell-snapshots, then rounded to multiples of 16."""
    rng = np.random.default_rng(seed)
    ni = rng.uniform(64, 512, n_blocks)
    nj = rng.uniform(32, 128, n_blocks)
    nh = rng.integers(1, 5, n_blocks)
    ns = 2 * nh + 1
    for _ in range(50):
        f = math.sqrt(target / float((ni * nj * ns).sum()))
        ni = np.clip(ni * f, 64, 512)
        nj = np.clip(nj * f, 32, 128)
    ni = np.clip(np.round(ni / 16) * 16, 64, 512).astype(int)
    nj = np.clip(np.round(nj / 16) * 16, 32, 128).astype(int)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ni, nj, nh)]


def make_problem(name: str) -> Problem:
    """The workloads (names describe what they are):

    cyl64x32_nh1      O-grid 64x32 around a unit circle, N_H=1, 100 iterations, FP64
    naca4blk_nh2      4 glued blocks of one C-grid (256x64, 128x64, 64x64 in the
                      bottom layer, 192x96 above the last two; c_grid_l), N_H=2,
                      500 iterations, FP64
    naca1024x512_nh4  C-grid 1024x512, N_H=4, FP32 bulk vs FP64 (converged forces)
    naca256x128_hh64  C-grid 256x128, N_H=2, 64 Hicks-Henne bumps + inflow angle (adjoint)
    batch32_mixed     32 O-grid blocks of uneven size, N_H in 1..4, about 8M
                      cell-snapshots, FP32 bulk, 1000 iterations
    Small variants for fast tests: cyl_tiny, naca_tiny, batch_tiny, and
    naca_tiny_hh8 (C-grid 64x16, N_H=1, 8 Hicks-Henne bumps) for converged
    total gradients.
    """
    if name == "cyl64x32_nh1":
        return Problem(name, [o_block(64, 32, 1)], flow_cylinder(), Solver(cfl=1.5), 100, 1304)
    if name == "naca4blk_nh2":
        blocks, cuts = c_grid_l(2)
        return Problem(name, blocks, flow_airfoil(), Solver(), 500, 1305, cuts=cuts)
    if name == "naca1024x512_nh4":
        return Problem(name, [c_block(1024, 512, 4)], flow_airfoil(), Solver(precision=1),
                       100000, 1306)
    if name == "naca256x128_hh64":
        rng = np.random.default_rng(1307)
        beta = rng.normal(0.0, 5e-4, 64)
        xy, dxy = hicks_henne_grid(256, 128, beta)
        p = Problem(name, [c_block(256, 128, 2, 0, xy)], flow_airfoil(), Solver(), 0, 1307)
        p.design = {"beta": beta, "dxy": dxy}
        return p
    if name == "batch32_mixed":
        draw = cfg5_draw()
        blocks = [o_block(a, b, c, k) for k, (a, b, c) in enumerate(draw)]
        return Problem(name, blocks, flow_cylinder(), Solver(precision=1), 1000, 1308)
    # small variants for fast tests (several tiles and ragged tails)
    if name == "cyl_tiny":
        return Problem(name, [o_block(40, 20, 1)], flow_cylinder(), Solver(cfl=1.5), 5, 11)
    if name == "naca_tiny":
        return Problem(name, [c_block(72, 20, 2)], flow_airfoil(), Solver(), 5, 12)
    if name == "naca_tiny_hh8":
        rng = np.random.default_rng(17)
        beta = rng.normal(0.0, 5e-4, 8)
        xy, dxy = hicks_henne_grid(64, 16, beta)
        p = Problem(name, [c_block(64, 16, 1, 0, xy)], flow_airfoil(), Solver(), 0, 17)
        p.design = {"beta": beta, "dxy": dxy}
        return p
    if name == "batch_tiny":
        blocks = [o_block(48, 18, 1, 0), c_block(76, 22, 2, 1), o_block(36, 40, 3, 2),
                  o_block(20, 12, 4, 3)]
        return Problem(name, blocks, flow_cylinder(), Solver(), 3, 13)
    raise KeyError(name)


WORKLOADS = ["cyl64x32_nh1", "naca4blk_nh2", "naca1024x512_nh4", "naca256x128_hh64",
             "batch32_mixed"]
