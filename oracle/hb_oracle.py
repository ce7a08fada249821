"""FP64 CPU oracle of the harmonic-balance (HB) Navier-Stokes residual and
its explicit Runge-Kutta pseudo-time iteration.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code
with the HIP library (no kernels, headers, tables or helpers) and imports
nothing from it; inputs (grids, initial states) come in as plain arrays.

It is plain, slow and meant to be read against the method:  every function
says which part of the method it follows.  The paper (Jackson & Campobasso,
COSA HB solver) describes the code structure but not the numerics: its HB
formulation section is missing, so the spatial scheme is the textbook
reading listed with each function (Roe flux with MUSCL/van Albada
reconstruction, diamond-path central viscous flux, time-collocation HB
operator, four-stage Runge-Kutta with local time stepping).

Parity status of each function (how it is pinned is in tests/test_oracle_*):
  hb_matrix, metrics, primitives, van_albada, roe_flux, diamond_gradient,
  residual (freestream, telescoping, block/shift symmetries), rk_iterate
  (scalar-ODE closed form, HB vs time-domain march), forces (closure,
  symmetry).  All are pinned; none is "parity unpinned".

Array conventions (paper §MPI Optimisations, halo pseudo code: the state is
q(i, j, ipde, n) with i fastest): one block's state is a tensor
q[n][v][j][i] (snapshot, conserved variable, row, column), FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

DT = torch.float64
WALL, FARFIELD, PERIODIC, CUT, WAKECUT, CUT_WALL, CUT_FARFIELD = 1, 2, 3, 4, 5, 6, 7
# sides glued by cut segments: CUT (covered exactly once), or partly glued
# with the rest of the side a wall (CUT_WALL) or far field (CUT_FARFIELD)
GLUED = (CUT, CUT_WALL, CUT_FARFIELD)


# ---------------------------------------------------------------------------
# Problem description (mirrors the C-ABI arguments; plain data only)
# ---------------------------------------------------------------------------
@dataclass
class OFlow:
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
        # reduced frequency k = omega * L / (2 |V_inf|)  ->  omega = 2 k M / L
        return 2.0 * self.k_red * self.mach / self.l_ref

    @property
    def mu(self) -> float:
        # Re = rho_inf |V_inf| L / mu with rho_inf = 1, |V_inf| = M
        return self.mach * self.l_ref / self.reynolds


@dataclass
class OSolver:
    cfl: float = 1.5
    rk_alpha: Tuple[float, ...] = (0.25, 1.0 / 3.0, 0.5, 1.0)
    entropy_delta: float = 0.1
    limiter_eps: float = 1e-12


@dataclass
class OBlock:
    ni: int
    nj: int
    n_harm: int
    xy: torch.Tensor                    # [2][nj+1][ni+1]
    bc: Tuple[int, int, int, int]       # imin, imax, jmin, jmax
    wake_ncells: int = 0
    body_id: int = 0

    @property
    def ns(self) -> int:
        return 2 * self.n_harm + 1


def from_synth(problem) -> Tuple[List[OBlock], OFlow, OSolver]:
    """Copy a synthetic problem description into the oracle's own types."""
    f, s = problem.flow, problem.solver
    flow = OFlow(f.mach, f.reynolds, f.prandtl, f.gamma, f.alpha0, f.alpha_amp, f.k_red,
                 f.l_ref, f.x_mom, f.y_mom)
    solver = OSolver(s.cfl, tuple(s.rk_alpha), s.entropy_delta, s.limiter_eps)
    blocks = [OBlock(b.ni, b.nj, b.n_harm, torch.as_tensor(b.xy, dtype=DT), tuple(b.bc),
                     b.wake_ncells, b.body_id) for b in problem.blocks]
    return blocks, flow, solver


def split(blocks: Sequence[OBlock], q: torch.Tensor) -> List[torch.Tensor]:
    out, o = [], 0
    for b in blocks:
        n = b.ns * 4 * b.nj * b.ni
        out.append(q[o:o + n].reshape(b.ns, 4, b.nj, b.ni))
        o += n
    return out


def join(parts: Sequence[torch.Tensor]) -> torch.Tensor:
    return torch.cat([p.reshape(-1) for p in parts])


# ---------------------------------------------------------------------------
# HB operator
# ---------------------------------------------------------------------------
def hb_matrix(n_harm: int, omega: float) -> torch.Tensor:
    """Spectral time-derivative operator of the time-collocation HB method.

    The paper's snapshots are n = 0..2*nharms (§MPI Optimisations, loops
    `do n = 0, 2*nharms`); it states no formula (its HB section is missing).
    Reading: snapshot n sits at t_n = n T / N_s, N_s = 2 N_H + 1, and the
    periodic signal is the trigonometric interpolant of degree N_H through
    the snapshots.  Differentiating the interpolant's cardinal functions at
    t_n gives  D[n][m] = (2 omega / N_s) * sum_{k=1..N_H} k sin(2 pi k (m-n) / N_s).
    """
    ns = 2 * n_harm + 1
    D = torch.zeros(ns, ns, dtype=DT)
    for n in range(ns):
        for m in range(ns):
            s = 0.0
            for k in range(1, n_harm + 1):
                s += k * math.sin(2.0 * math.pi * k * (m - n) / ns)
            D[n, m] = 2.0 * omega / ns * s
    return D


def snapshot_alpha(flow: OFlow, ns: int) -> torch.Tensor:
    """Incidence of each snapshot: alpha(t_n) = alpha0 + A sin(omega t_n),
    omega t_n = 2 pi n / N_s."""
    n = torch.arange(ns, dtype=DT)
    return flow.alpha0 + flow.alpha_amp * torch.sin(2.0 * math.pi * n / ns)


def freestream_prim(flow: OFlow, ns: int, alpha0: Optional[torch.Tensor] = None
                    ) -> torch.Tensor:
    """Free-stream primitives (rho, u, v, p) per snapshot, [ns][4].
    Non-dimensionalisation: rho_inf = 1, c_inf = 1, p_inf = 1/gamma, |V| = M.
    `alpha0` may be a 0-d tensor (so that autograd can differentiate)."""
    a0 = flow.alpha0 if alpha0 is None else alpha0
    n = torch.arange(ns, dtype=DT)
    alpha = a0 + flow.alpha_amp * torch.sin(2.0 * math.pi * n / ns)
    one = torch.ones(ns, dtype=DT)
    return torch.stack([one, flow.mach * torch.cos(alpha), flow.mach * torch.sin(alpha),
                        one / flow.gamma], dim=1)


# ---------------------------------------------------------------------------
# Metrics
# ---------------------------------------------------------------------------
def metrics(xy: torch.Tensor):
    """Finite-volume metrics of a structured block (nodes xy[2][nj+1][ni+1]).

    S_I(i,j): normal of the edge node(i,j) -> node(i,j+1), (dy, -dx), length
              = edge length, pointing towards +i.           shape [nj][ni+1][2]
    S_J(i,j): normal of the edge node(i,j) -> node(i+1,j), (-dy, dx), pointing
              towards +j.                                    shape [nj+1][ni][2]
    V(i,j):   cell area, half the cross product of the diagonals.  [nj][ni]
    C(i,j):   cell centre, mean of the four nodes.                [nj][ni][2]
    """
    x, y = xy[0], xy[1]
    SI = torch.stack([y[1:, :] - y[:-1, :], -(x[1:, :] - x[:-1, :])], dim=-1)
    SJ = torch.stack([-(y[:, 1:] - y[:, :-1]), x[:, 1:] - x[:, :-1]], dim=-1)
    x1, y1 = x[:-1, :-1], y[:-1, :-1]
    x2, y2 = x[:-1, 1:], y[:-1, 1:]
    x3, y3 = x[1:, 1:], y[1:, 1:]
    x4, y4 = x[1:, :-1], y[1:, :-1]
    V = 0.5 * ((x3 - x1) * (y4 - y2) - (y3 - y1) * (x4 - x2))
    C = torch.stack([(x1 + x2 + x3 + x4) / 4.0, (y1 + y2 + y3 + y4) / 4.0], dim=-1)
    return SI, SJ, V, C


# ---------------------------------------------------------------------------
# Thermodynamics
# ---------------------------------------------------------------------------
def primitives(q: torch.Tensor, gamma: float) -> torch.Tensor:
    """Conserved (rho, rho u, rho v, rho E) -> primitive (rho, u, v, p),
    perfect gas.  q[..., 4, ...] with the variable on dim -3."""
    rho = q[..., 0, :, :]
    u = q[..., 1, :, :] / rho
    v = q[..., 2, :, :] / rho
    p = (gamma - 1.0) * (q[..., 3, :, :] - 0.5 * rho * (u * u + v * v))
    return torch.stack([rho, u, v, p], dim=-3)


def mirror_prim(w: torch.Tensor) -> torch.Tensor:
    """No-slip adiabatic wall ghost: same rho and p, velocity reversed."""
    return torch.stack([w[..., 0, :, :], -w[..., 1, :, :], -w[..., 2, :, :],
                        w[..., 3, :, :]], dim=-3)


# ---------------------------------------------------------------------------
# Ghost cells (two layers per side; the paper's "cuts" are block-edge halos)
# ---------------------------------------------------------------------------
def side_length(b: OBlock, side: int) -> int:
    """Cells along side 0..3 = imin, imax, jmin, jmax (positions are j on the
    i sides, i on the j sides)."""
    return b.nj if side < 2 else b.ni


def cut_partners(blocks: Sequence[OBlock], cuts) -> dict:
    """(block, side) -> the segments gluing that side, sorted by start: each
    (start, length, partner block, partner side, partner start, reversed).

    A cut joins block edges (the paper's "cuts" between blocks, whose halos
    are exchanged every Runge-Kutta step; §MPI Optimisations sends a cut as a
    sequence of sections along a block's boundary).  Read here as a segment
    of `length` cells of one side glued to a segment of another side (any
    two sides, possibly of the same block), cell start_a + t against
    start_b + t, or start_b + length - 1 - t when reversed.  A cut is
    (a, side_a, start_a, b, side_b, start_b, length, reversed), or
    (a, side_a, b, side_b[, reversed]) for two whole sides of equal length.
    Every side of kind CUT must be covered by its segments exactly once; a
    side of kind CUT_WALL or CUT_FARFIELD at most once (a block edge made of
    sections of which some are glued and the rest are wall or far field);
    glued blocks share n_harm.  Sides are numbered 0..3 = imin, imax, jmin,
    jmax."""
    m = {}
    for c in cuts:
        c = tuple(int(x) for x in c)
        if len(c) in (4, 5):
            a, sa, b, sb = c[:4]
            la, lb = side_length(blocks[a], sa), side_length(blocks[b], sb)
            if la != lb:
                raise ValueError("whole-side cuts need sides of equal length")
            c = (a, sa, 0, b, sb, 0, la, c[4] if len(c) == 5 else 0)
        if len(c) != 8:
            raise ValueError("a cut has 4, 5 or 8 entries")
        a, sa, st_a, b, sb, st_b, ln, rev = c
        A, B = blocks[a], blocks[b]
        if A.bc[sa] not in GLUED or B.bc[sb] not in GLUED or A.n_harm != B.n_harm:
            raise ValueError("cut sides must be of a glued kind with equal n_harm")
        if ln < 1 or st_a < 0 or st_b < 0 or st_a + ln > side_length(A, sa) \
                or st_b + ln > side_length(B, sb):
            raise ValueError("a cut segment leaves its side")
        m.setdefault((a, sa), []).append((st_a, ln, b, sb, st_b, 1 if rev else 0))
        m.setdefault((b, sb), []).append((st_b, ln, a, sa, st_a, 1 if rev else 0))
    for key in m:
        m[key].sort()
    for k, blk in enumerate(blocks):
        for side in range(4):
            if blk.bc[side] not in GLUED:
                continue
            pos = 0
            for st, ln, *_ in m.get((k, side), []):
                if st < pos or (blk.bc[side] == CUT and st != pos):
                    raise ValueError("the cut segments of a side must cover it exactly once")
                pos = st + ln
            if blk.bc[side] == CUT and pos != side_length(blk, side):
                raise ValueError("a CUT side is not covered by its cuts")
    return m


def cut_segment(blocks: Sequence[OBlock], cutmap: dict, b: int, side: int, p: int):
    """The segment of side `side` of block b that covers position p (a
    position beyond the side's ends counts as its end cell), or None."""
    L = side_length(blocks[b], side)
    pc = min(max(p, 0), L - 1)
    for g in cutmap.get((b, side), []):
        if g[0] <= pc < g[0] + g[1]:
            return g
    return None


def cut_cell(blocks: Sequence[OBlock], cutmap: dict, b: int, side: int, k: int, p: int):
    """The cell across a cut from ghost layer k (0 nearest) at position p of
    side `side` of block b: (block, i, j) at depth k inside the partner side.
    A position beyond the side's ends (a corner ghost) continues the mapping
    of the end segment; the result may then lie outside the partner, where
    the partner's own side rules apply."""
    st, ln, a, sa, st_a, rev = cut_segment(blocks, cutmap, b, side, p)
    t = p - st
    pp = st_a + (ln - 1 - t if rev else t)
    A = blocks[a]
    if sa == 0:
        return a, k, pp
    if sa == 1:
        return a, A.ni - 1 - k, pp
    if sa == 2:
        return a, pp, k
    return a, pp, A.nj - 1 - k


def resolve_ghost(blocks: Sequence[OBlock], cutmap: dict, b: int, i: int, j: int, wall=None):
    """Where ghost-extended cell (i, j) of block b takes its value from:
    (block, i, j, mirror) of an interior cell, or (block, None, None,
    mirror) for the free stream; mirror = parity of the wall images met.
    With `wall` a list, the wall faces met are appended to it as (block,
    side, position along the side).
    The i sides are resolved first, then the j sides (the order that
    defines the corner ghosts; on grids without cuts either order gives the
    same cells, and with the i sides first a C-grid cut into wake and
    airfoil blocks keeps the single block's ghosts at the trailing edge);
    across a cut the partner block's own rules apply to what is still
    outside it.  On a partly glued side the cells no segment covers follow
    the side's rest kind (wall or far field)."""
    mir = 0
    for _ in range(8):
        B = blocks[b]
        if i < 0 or i >= B.ni:
            side = 0 if i < 0 else 1
            k = -1 - i if i < 0 else i - B.ni
            kind = B.bc[side]
            if kind == PERIODIC:
                i = i % B.ni
            elif kind in GLUED and cut_segment(blocks, cutmap, b, side, j) is not None:
                b, i, j = cut_cell(blocks, cutmap, b, side, k, j)
            elif kind in (WALL, CUT_WALL):
                if wall is not None:
                    wall.append((b, side, j))
                i = k if side == 0 else B.ni - 1 - k
                mir ^= 1
            elif kind in (FARFIELD, CUT_FARFIELD):
                return b, None, None, mir
            else:
                raise ValueError("unsupported i-side boundary %d" % kind)
            continue
        if j < 0 or j >= B.nj:
            side = 2 if j < 0 else 3
            k = -1 - j if j < 0 else j - B.nj
            kind = B.bc[side]
            if kind == PERIODIC:
                j = j % B.nj
            elif kind == WAKECUT and side == 2 and (i < B.wake_ncells or i >= B.ni - B.wake_ncells):
                i, j = B.ni - 1 - i, k
            elif kind in GLUED and cut_segment(blocks, cutmap, b, side, i) is not None:
                b, i, j = cut_cell(blocks, cutmap, b, side, k, i)
            elif kind in (WALL, CUT_WALL) or (kind == WAKECUT and side == 2):
                if wall is not None:
                    wall.append((b, side, i))
                j = k if side == 2 else B.nj - 1 - k
                mir ^= 1
            elif kind in (FARFIELD, CUT_FARFIELD):
                return b, None, None, mir
            else:
                raise ValueError("unsupported j-side boundary %d" % kind)
            continue
        return b, i, j, mir
    raise ValueError("ghost resolution does not end (cuts around a singular corner)")


_GHOST_MAPS = {}


def ghost_map(blocks, cutmap, k: int) -> dict:
    """resolve_ghost for every ghost cell of block k, grouped by source:
    (source block, far field?, mirror) -> index tensors (je, ie, sj, si) of
    the ghost cells (ghost-extended indices) and of their source cells (0
    for the far field).  The map depends only on the grid's topology and is
    kept per topology."""
    key = (k, tuple((b.ni, b.nj, tuple(b.bc), b.wake_ncells) for b in blocks),
           tuple(sorted((kk, tuple(v)) for kk, v in cutmap.items())))
    if key not in _GHOST_MAPS:
        b = blocks[k]
        groups = {}
        for je in range(b.nj + 4):
            for ie in range(b.ni + 4):
                i, j = ie - 2, je - 2
                if 0 <= i < b.ni and 0 <= j < b.nj:
                    continue
                src, si, sj, mir = resolve_ghost(blocks, cutmap, k, i, j)
                g = groups.setdefault((src, si is None, mir), ([], [], [], []))
                g[0].append(je)
                g[1].append(ie)
                g[2].append(0 if si is None else sj)
                g[3].append(0 if si is None else si)
        _GHOST_MAPS[key] = {kk: tuple(torch.tensor(x, dtype=torch.long) for x in v)
                            for kk, v in groups.items()}
    return _GHOST_MAPS[key]


_WALL_MAPS = {}


def wall_map(blocks, cutmap, k: int) -> list:
    """The ghost cells of block k that are wall images: (je, ie, block,
    side, position) with the wall face their resolution mirrored at
    (resolve_ghost)."""
    key = (k, tuple((b.ni, b.nj, tuple(b.bc), b.wake_ncells) for b in blocks),
           tuple(sorted((kk, tuple(v)) for kk, v in cutmap.items())))
    if key not in _WALL_MAPS:
        b = blocks[k]
        out = []
        for je in range(b.nj + 4):
            for ie in range(b.ni + 4):
                i, j = ie - 2, je - 2
                if 0 <= i < b.ni and 0 <= j < b.nj:
                    continue
                walls = []
                resolve_ghost(blocks, cutmap, k, i, j, walls)
                if len(walls) > 1:
                    raise ValueError("a ghost meets more than one wall")
                if walls:
                    out.append((je, ie) + walls[0])
        _WALL_MAPS[key] = out
    return _WALL_MAPS[key]


def extend_cut(blocks, ws, winfs, cutmap, k: int) -> torch.Tensor:
    """Ghost-extended primitives [ns][4][nj+4][ni+4] of block k, which has
    glued sides: every ghost cell from resolve_ghost (ghost_map), taken from
    the blocks' interior fields of the same snapshots (Jacobi exchange)."""
    b = blocks[k]
    w = ws[k]
    ns = w.shape[0]
    we = torch.zeros(ns, 4, b.nj + 4, b.ni + 4, dtype=w.dtype)
    we[:, :, 2:b.nj + 2, 2:b.ni + 2] = w
    for (src, ff, mir), (je, ie, sj, si) in ghost_map(blocks, cutmap, k).items():
        if ff:
            v = winfs[src][:, :, None].expand(ns, 4, len(je))
        else:
            v = ws[src][:, :, sj, si]
        if mir:
            v = mirror_prim(v[..., None])[..., 0]
        we[:, :, je, ie] = v
    return we


def cut_ghost_centres(blocks, cutmap, Cs, k: int) -> dict:
    """Centres [L][2] of the first ghost layer of each glued side of block k:
    the centres (Cs[block][j, i]) of the cells across the cut; NaN for the
    cells of a partly glued side that no segment covers (their ghost centre
    is the mirrored one, ghost_centres)."""
    b = blocks[k]
    out = {}
    nan = torch.full((2,), float("nan"), dtype=DT)
    for side in range(4):
        if b.bc[side] not in GLUED:
            continue
        cs = []
        for p in range(side_length(b, side)):
            if cut_segment(blocks, cutmap, k, side, p) is None:
                cs.append(nan)
                continue
            a, i, j = cut_cell(blocks, cutmap, k, side, 0, p)
            cs.append(Cs[a][j, i])
        out[side] = torch.stack(cs)
    return out


def extend_i(b: OBlock, w: torch.Tensor, winf: torch.Tensor, nbr=None) -> torch.Tensor:
    """Ghost columns of the i sides: w[ns][4][nj][ni] -> [ns][4][nj][ni+4]
    (cell i at column i+2).  `nbr` maps a CUT side (0 or 1) to the
    neighbour block's interior field."""
    ns, _, nj, ni = w.shape
    ff = winf[:, :, None, None]
    cols = [None] * (ni + 4)
    for k in range(ni):
        cols[k + 2] = w[..., k]
    for side in (0, 1):
        kind = b.bc[side]
        for k in (0, 1):                       # ghost layer k
            gi = -1 - k if side == 0 else ni + k
            if kind == PERIODIC:
                c = w[..., gi % ni]
            elif kind == FARFIELD:
                c = ff[..., 0].expand(ns, 4, nj)
            elif kind == WALL:
                src = k if side == 0 else ni - 1 - k
                c = mirror_prim(w[..., src:src + 1])[..., 0]
            elif kind == CUT:
                wa = nbr[side]                 # glued to the other block's imax / imin
                c = wa[..., wa.shape[-1] - 1 - k] if side == 0 else wa[..., k]
            else:
                raise ValueError("unsupported i-side boundary %d" % kind)
            cols[gi + 2] = c
    return torch.stack(cols, dim=-1)


def extend_j(b: OBlock, wi: torch.Tensor, winf: torch.Tensor, nbr=None) -> torch.Tensor:
    """Ghost rows of the j sides over the i-extended rows wi[ns][4][nj][ni+4]
    -> [ns][4][nj+4][ni+4]; this also defines the corner ghosts.  `nbr` maps
    a CUT side (2 or 3) to the neighbour block's i-extended field."""
    ns, _, nj, nie = wi.shape
    ni = nie - 4
    ff = winf[:, :, None, None]
    rows = [None] * (nj + 4)
    for k in range(nj):
        rows[k + 2] = wi[..., k, :]
    for side in (2, 3):
        kind = b.bc[side]
        for k in (0, 1):
            gj = -1 - k if side == 2 else nj + k
            src = k if side == 2 else nj - 1 - k
            if kind == PERIODIC:
                r = wi[..., gj % nj, :]
            elif kind == FARFIELD:
                r = ff[..., 0, 0, None].expand(ns, 4, ni + 4)
            elif kind == WALL:
                r = mirror_prim(wi[..., src:src + 1, :])[..., 0, :]
            elif kind == WAKECUT and side == 2:
                wall = mirror_prim(wi[..., src:src + 1, :])[..., 0, :]
                parts = []
                for ie in range(ni + 4):
                    i = ie - 2
                    if i < b.wake_ncells or i >= ni - b.wake_ncells:
                        parts.append(wi[..., src, (ni - 1 - i) + 2])
                    else:
                        parts.append(wall[..., ie])
                r = torch.stack(parts, dim=-1)
            elif kind == CUT:
                wa = nbr[side]
                r = wa[..., wa.shape[-2] - 1 - k, :] if side == 2 else wa[..., k, :]
            else:
                raise ValueError("unsupported j-side boundary %d" % kind)
            rows[gj + 2] = r
    return torch.stack(rows, dim=-2)


def extend(b: OBlock, w: torch.Tensor, winf: torch.Tensor) -> torch.Tensor:
    """Primitive field w[ns][4][nj][ni] -> ghost-extended we[ns][4][nj+4][ni+4]
    (cell (i, j) at index (j+2, i+2)) of a block without cuts.

    Rules (the paper gives none; reading):
      periodic:  copy of the cells one period away;
      farfield:  both layers = free stream of the snapshot's incidence;
      wall:      ghost k (k = 0 nearest) mirrors interior cell k;
      wake cut:  C-grid jmin: ghost (i, -1-k) = cell (ni-1-i, k) for i in the
                 wake (i < wake_ncells or i >= ni - wake_ncells), wall otherwise;
      cut:       the glued block's cells (extend_all).
    The i sides are filled first (rows 0..nj-1); the j sides then apply their
    rule to the i-extended rows, which also defines the corner ghosts.
    """
    we = extend_j(b, extend_i(b, w, winf), winf)
    # the i sides come first, and the far field ends a ghost's resolution:
    # the corner ghosts beside a far-field i side are free stream
    for side, cols in ((0, slice(0, 2)), (1, slice(b.ni + 2, b.ni + 4))):
        if b.bc[side] == FARFIELD:
            for rows in (slice(0, 2), slice(b.nj + 2, b.nj + 4)):
                we[:, :, rows, cols] = winf[:, :, None, None]
    return we


def extend_all(blocks, ws, winfs, cutmap):
    """Ghost-extended primitive fields of all blocks.  A cut ghost is a cell
    of the glued block taken from the same input (Jacobi exchange); blocks
    without glued sides use extend()."""
    return [extend_cut(blocks, ws, winfs, cutmap, k) if any(s in GLUED for s in b.bc)
            else extend(b, w, wf) for k, (b, w, wf) in enumerate(zip(blocks, ws, winfs))]


def reflect(p: torch.Tensor, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Mirror image of point p across the line through a and b (last dim 2)."""
    e = b - a
    t = ((p - a) * e).sum(-1, keepdim=True) / (e * e).sum(-1, keepdim=True)
    foot = a + t * e
    return 2.0 * foot - p


def ghost_centres(b: OBlock, xy: torch.Tensor, C: torch.Tensor, nbrC=None):
    """Centres of the first ghost layer on each side (for the viscous diamond
    of boundary faces).  Periodic, wake-cut and cut ghosts are real cells, so
    their centre is the partner cell's centre (`nbrC` maps a glued side to
    the centres [L][2] of the cells across it, cut_ghost_centres, NaN where
    no segment covers the cell); wall and farfield ghost centres are the
    interior centre mirrored across the boundary face.
    Returns (c_imin [nj][2], c_imax [nj][2], c_jmin [ni][2], c_jmax [ni][2])."""
    nj, ni = C.shape[0], C.shape[1]
    P = xy.permute(1, 2, 0)                   # nodes [nj+1][ni+1][2]
    out = []
    for side in range(4):
        kind = b.bc[side]
        if side == 0:
            real = C[:, ni - 1]
            mir = reflect(C[:, 0], P[:-1, 0], P[1:, 0])
        elif side == 1:
            real = C[:, 0]
            mir = reflect(C[:, ni - 1], P[:-1, ni], P[1:, ni])
        elif side == 2:
            real = C[nj - 1, :]
            mir = reflect(C[0, :], P[0, :-1], P[0, 1:])
        else:
            real = C[0, :]
            mir = reflect(C[nj - 1, :], P[nj, :-1], P[nj, 1:])
        if kind == PERIODIC:
            out.append(real)
        elif kind in GLUED:
            c = nbrC[side]
            out.append(torch.where(torch.isnan(c), mir, c))
        elif kind in (WALL, FARFIELD):
            out.append(mir)
        elif kind == WAKECUT:
            i = torch.arange(ni)
            wake = (i < b.wake_ncells) | (i >= ni - b.wake_ncells)
            partner = C[0, ni - 1 - i]
            out.append(torch.where(wake[:, None], partner, mir))
        else:
            raise ValueError(kind)
    return tuple(out)


# ---------------------------------------------------------------------------
# Reconstruction and fluxes
# ---------------------------------------------------------------------------
def van_albada(a: torch.Tensor, b: torch.Tensor, eps: float) -> torch.Tensor:
    """Van Albada limited slope  (a+b)(ab+eps)/(a^2+b^2+2 eps)."""
    return (a + b) * (a * b + eps) / (a * a + b * b + 2.0 * eps)


def muscl(wm2, wm1, wp0, wp1, eps):
    """MUSCL face states between cells m1 and p0 from the four cells on the
    grid line (index-space slopes, van Albada limiter on primitives)."""
    wl = wm1 + 0.5 * van_albada(wm1 - wm2, wp0 - wm1, eps)
    wr = wp0 - 0.5 * van_albada(wp0 - wm1, wp1 - wp0, eps)
    return wl, wr


def euler_normal_flux(w: torch.Tensor, nx, ny, gamma):
    """Inviscid flux through a unit normal (nx, ny); w = (rho, u, v, p) on
    dim 0."""
    rho, u, v, p = w[0], w[1], w[2], w[3]
    qn = u * nx + v * ny
    rhoE = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return torch.stack([rho * qn, rho * u * qn + p * nx, rho * v * qn + p * ny,
                        (rhoE + p) * qn])


def conserved(w: torch.Tensor, gamma: float) -> torch.Tensor:
    """(rho, u, v, p) on dim 0 -> (rho, rho u, rho v, rho E) on dim 0."""
    rho, u, v, p = w[0], w[1], w[2], w[3]
    return torch.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def roe_flux(wl: torch.Tensor, wr: torch.Tensor, S: torch.Tensor, gamma: float,
             delta_frac: float, vg: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Roe's approximate Riemann solver (textbook form) times the face length.

    wl, wr: primitives with the variable on dim 0; S: face normal vector with
    its components on dim 0 (length = face length), pointing from L to R.
    Roe averages use sqrt(rho) weights.  The waves are the two acoustic waves
    (q_n -/+ c), the entropy wave and the shear wave (both q_n).  Harten's
    entropy fix on the acoustic eigenvalues: |l| -> (l^2 + d^2)/(2 d) when
    |l| < d, d = delta_frac * c~ (delta_frac = 0 switches it off).
    F = |S| [ (F(L) + F(R))/2 - (1/2) sum_k |l_k| a_k r_k ].

    Moving face (arbitrary Lagrangian-Eulerian form): vg = x_t . S, the
    face's grid velocity times its length-weighted normal.  The flux through
    the moving face is F.n - (vg/|S|) U, and every eigenvalue is measured
    relative to the face, q_n - vg/|S| (the eigenvectors do not change).
    vg = None is the fixed face.
    """
    area = torch.sqrt(S[0] * S[0] + S[1] * S[1])
    nx, ny = S[0] / area, S[1] / area
    g = gamma
    rl, ul, vl, pl = wl[0], wl[1], wl[2], wl[3]
    rr, ur, vr, pr = wr[0], wr[1], wr[2], wr[3]
    hl = g / (g - 1.0) * pl / rl + 0.5 * (ul * ul + vl * vl)
    hr = g / (g - 1.0) * pr / rr + 0.5 * (ur * ur + vr * vr)
    sl, sr = torch.sqrt(rl), torch.sqrt(rr)
    rt = sl * sr
    ut = (sl * ul + sr * ur) / (sl + sr)
    vt = (sl * vl + sr * vr) / (sl + sr)
    ht = (sl * hl + sr * hr) / (sl + sr)
    q2t = ut * ut + vt * vt
    ct = torch.sqrt((g - 1.0) * (ht - 0.5 * q2t))
    qnt = ut * nx + vt * ny
    qrel = qnt if vg is None else qnt - vg / area
    dr, du, dv, dp = rr - rl, ur - ul, vr - vl, pr - pl
    dqn = du * nx + dv * ny
    # wave strengths
    a1 = (dp - rt * ct * dqn) / (2.0 * ct * ct)
    a4 = (dp + rt * ct * dqn) / (2.0 * ct * ct)
    a2 = dr - dp / (ct * ct)
    l1 = torch.abs(qrel - ct)
    l4 = torch.abs(qrel + ct)
    l2 = torch.abs(qrel)
    if delta_frac > 0.0:
        d = delta_frac * ct
        l1 = torch.where(l1 < d, (l1 * l1 + d * d) / (2.0 * d), l1)
        l4 = torch.where(l4 < d, (l4 * l4 + d * d) / (2.0 * d), l4)
    one = torch.ones_like(ut)
    zero = torch.zeros_like(ut)
    r1 = torch.stack([one, ut - ct * nx, vt - ct * ny, ht - qnt * ct])
    r4 = torch.stack([one, ut + ct * nx, vt + ct * ny, ht + qnt * ct])
    r2 = torch.stack([one, ut, vt, 0.5 * q2t])
    shear = rt * torch.stack([zero, du - nx * dqn, dv - ny * dqn,
                              ut * du + vt * dv - qnt * dqn])
    diss = l1 * a1 * r1 + l4 * a4 * r4 + l2 * (a2 * r2 + shear)
    fl = euler_normal_flux(wl, nx, ny, g)
    fr = euler_normal_flux(wr, nx, ny, g)
    if vg is not None:
        fl = fl - vg / area * conserved(wl, g)
        fr = fr - vg / area * conserved(wr, g)
    return area * (0.5 * (fl + fr) - 0.5 * diss)


def polygon_gradient(px: Sequence[torch.Tensor], py: Sequence[torch.Tensor],
                     phi: Sequence[torch.Tensor]):
    """Green-Gauss gradient of phi over a polygon (vertices in order), with
    trapezoidal edge values:  grad = (1/A) sum_e (phi_a + phi_b)/2 * n_e,
    n_e = (dy, -dx) of edge a->b, A = signed shoelace area.  Exact for linear
    phi on any non-degenerate polygon of either orientation."""
    k = len(px)
    gx = torch.zeros_like(phi[0])
    gy = torch.zeros_like(phi[0])
    area = torch.zeros_like(px[0])
    for a in range(k):
        b = (a + 1) % k
        pm = 0.5 * (phi[a] + phi[b])
        gx = gx + pm * (py[b] - py[a])
        gy = gy - pm * (px[b] - px[a])
        area = area + 0.5 * (px[a] * py[b] - px[b] * py[a])
    return gx / area, gy / area


def viscous_face_flux(wL, wR, nodeA, nodeB, cL, cR, pA, pB, S, flow: OFlow):
    """Central viscous flux through one face, times the face length.

    Gradients of (u, v, T), T = gamma p / rho, by Green-Gauss on the diamond
    (centre L, node A, centre R, node B); node values are given.  Face
    velocity = mean of L and R.  Constant viscosity mu = M L / Re, Stokes
    hypothesis (lambda = -2/3 mu), heat flux -mu/((gamma-1) Pr) grad T.
    wL, wR, nodeA, nodeB: primitives/values with the variable on dim 0 holding
    (u, v, T); c*, p*: points with components on dim 0; S: face normal.
    Returns the 4-vector (0, tau.S, energy) on dim 0."""
    mu = flow.mu
    kappa = mu / ((flow.gamma - 1.0) * flow.prandtl)
    px = [cL[0], pA[0], cR[0], pB[0]]
    py = [cL[1], pA[1], cR[1], pB[1]]
    grads = []
    for v in range(3):
        grads.append(polygon_gradient(px, py, [wL[v], nodeA[v], wR[v], nodeB[v]]))
    (ux, uy), (vx, vy), (tx, ty) = grads
    div = ux + vy
    txx = mu * (2.0 * ux - 2.0 / 3.0 * div)
    tyy = mu * (2.0 * vy - 2.0 / 3.0 * div)
    txy = mu * (uy + vx)
    uf = 0.5 * (wL[0] + wR[0])
    vf = 0.5 * (wL[1] + wR[1])
    fx = txx * S[0] + txy * S[1]
    fy = txy * S[0] + tyy * S[1]
    fe = uf * fx + vf * fy + kappa * (tx * S[0] + ty * S[1])
    return torch.stack([torch.zeros_like(fx), fx, fy, fe])


def uvt(w: torch.Tensor, gamma: float) -> torch.Tensor:
    """(rho, u, v, p) on dim -3 -> (u, v, T = gamma p / rho) on dim -3."""
    return torch.stack([w[..., 1, :, :], w[..., 2, :, :],
                        gamma * w[..., 3, :, :] / w[..., 0, :, :]], dim=-3)


# ---------------------------------------------------------------------------
# Residual of one block
# ---------------------------------------------------------------------------
def face_fluxes(b: OBlock, q: torch.Tensor, flow: OFlow, solver: OSolver,
                alpha0: Optional[torch.Tensor] = None, xy: Optional[torch.Tensor] = None,
                winf: Optional[torch.Tensor] = None, we: Optional[torch.Tensor] = None,
                nbrC=None, vg=None):
    """Net face fluxes (inviscid minus viscous, times face length) of every
    i-face FI[ns][4][nj][ni+1] and j-face FJ[ns][4][nj+1][ni] of one block,
    for all snapshots; q is the conserved state q[ns][4][nj][ni].  `winf`
    overrides the far-field primitives per snapshot ([ns][4]); a block with
    cuts passes its ghost-extended primitives `we` and the glued blocks'
    centres `nbrC` (extend_all).  `vg` = (vg_I [nj][ni+1], vg_J [nj+1][ni]):
    grid velocity times face normal of moving faces (roe_flux), None for a
    fixed grid."""
    g = flow.gamma
    vgi, vgj = (None, None) if vg is None else vg
    xy = b.xy if xy is None else xy
    SI, SJ, V, C = metrics(xy)
    ns, _, nj, ni = q.shape
    if we is None:
        w = primitives(q, g)
        if winf is None:
            winf = freestream_prim(flow, ns, alpha0)
        we = extend(b, w, winf)                       # [ns][4][nj+4][ni+4]
    eps = solver.limiter_eps
    # ---- inviscid: MUSCL along grid lines + Roe --------------------------
    # i-face i (0..ni) between cells i-1 and i, rows j = 0..nj-1
    row = we[:, :, 2:nj + 2, :]
    wl, wr = muscl(row[..., 0:ni + 1], row[..., 1:ni + 2], row[..., 2:ni + 3],
                   row[..., 3:ni + 4], eps)
    SIt = SI.permute(2, 0, 1)                         # [2][nj][ni+1]
    FI = roe_flux(wl.transpose(0, 1), wr.transpose(0, 1), SIt, g,
                  solver.entropy_delta, vgi).transpose(0, 1)
    col = we[:, :, :, 2:ni + 2]
    wl, wr = muscl(col[:, :, 0:nj + 1], col[:, :, 1:nj + 2], col[:, :, 2:nj + 3],
                   col[:, :, 3:nj + 4], eps)
    SJt = SJ.permute(2, 0, 1)                         # [2][nj+1][ni]
    FJ = roe_flux(wl.transpose(0, 1), wr.transpose(0, 1), SJt, g,
                  solver.entropy_delta, vgj).transpose(0, 1)
    # ---- viscous ---------------------------------------------------------
    t = uvt(we, g)                                    # [ns][3][nj+4][ni+4]
    # node (i, j), i = 0..ni, j = 0..nj: mean of cells (i-1..i, j-1..j)
    nodev = 0.25 * (t[:, :, 1:nj + 2, 1:ni + 2] + t[:, :, 1:nj + 2, 2:ni + 3]
                    + t[:, :, 2:nj + 3, 1:ni + 2] + t[:, :, 2:nj + 3, 2:ni + 3])
    cim, cip, cjm, cjp = ghost_centres(b, xy, C, nbrC)
    # extended centres for the cells L/R of i-faces: [nj][ni+2][2]
    ce_i = torch.cat([cim[:, None, :], C, cip[:, None, :]], dim=1)
    ce_j = torch.cat([cjm[None, :, :], C, cjp[None, :, :]], dim=0)   # [nj+2][ni][2]
    P = xy                                            # [2][nj+1][ni+1]
    # i-faces: L = (i-1, j), R = (i, j); A = node (i, j), B = node (i, j+1)
    tL = t[:, :, 2:nj + 2, 1:ni + 2]
    tR = t[:, :, 2:nj + 2, 2:ni + 3]
    nA = nodev[:, :, 0:nj, :]
    nB = nodev[:, :, 1:nj + 1, :]
    cL = ce_i[:, 0:ni + 1, :].permute(2, 0, 1)
    cR = ce_i[:, 1:ni + 2, :].permute(2, 0, 1)
    pA = P[:, 0:nj, :]
    pB = P[:, 1:nj + 1, :]
    GI = viscous_face_flux(tL.transpose(0, 1), tR.transpose(0, 1), nA.transpose(0, 1),
                           nB.transpose(0, 1), cL, cR, pA, pB, SIt, flow).transpose(0, 1)
    # j-faces: L = (i, j-1), R = (i, j); vertices L, B = node (i+1, j), R, A = node (i, j)
    tL = t[:, :, 1:nj + 2, 2:ni + 2]
    tR = t[:, :, 2:nj + 3, 2:ni + 2]
    nA = nodev[:, :, :, 0:ni]
    nB = nodev[:, :, :, 1:ni + 1]
    cL = ce_j[0:nj + 1].permute(2, 0, 1)
    cR = ce_j[1:nj + 2].permute(2, 0, 1)
    pA = P[:, :, 0:ni]
    pB = P[:, :, 1:ni + 1]
    GJ = viscous_face_flux(tL.transpose(0, 1), tR.transpose(0, 1), nB.transpose(0, 1),
                           nA.transpose(0, 1), cL, cR, pB, pA, SJt, flow).transpose(0, 1)
    return FI - GI, FJ - GJ


def spatial_residual(b, q, flow, solver, alpha0=None, xy=None, winf=None, we=None,
                     nbrC=None) -> torch.Tensor:
    """R(i,j) = F(i+1,j) - F(i,j) + G(i,j+1) - G(i,j): net outflow of the cell."""
    FI, FJ = face_fluxes(b, q, flow, solver, alpha0, xy, winf, we, nbrC)
    return (FI[..., :, 1:] - FI[..., :, :-1]) + (FJ[..., 1:, :] - FJ[..., :-1, :])


def hb_source(b: OBlock, q: torch.Tensor, flow: OFlow, xy=None) -> torch.Tensor:
    """V (D Q)_n: the cell volume times the HB time derivative of the
    conserved state at snapshot n (couples the snapshots pointwise)."""
    xy = b.xy if xy is None else xy
    V = metrics(xy)[2]
    D = hb_matrix(b.n_harm, flow.omega)
    dq = torch.einsum("nm,mvji->nvji", D, q)
    return V * dq


def residual(b, q, flow, solver, alpha0=None, xy=None, we=None, nbrC=None) -> torch.Tensor:
    """HB residual R*_n = R(Q_n) + V (D Q)_n of one block.  The pseudo-time
    system is V dQ/dtau = -R*."""
    return (spatial_residual(b, q, flow, solver, alpha0, xy, None, we, nbrC)
            + hb_source(b, q, flow, xy))


def _halos(blocks, qs, flow, cuts, alpha0=None, xys=None):
    """Ghost-extended primitives and glued-block centres of all blocks, or
    (None, None) per block when there are no cuts."""
    if not cuts:
        return [None] * len(blocks), [None] * len(blocks)
    xys = [b.xy for b in blocks] if xys is None else xys
    P = cut_partners(blocks, cuts)
    ws = [primitives(qb, flow.gamma) for qb in qs]
    winfs = [freestream_prim(flow, b.ns, alpha0) for b in blocks]
    wes = extend_all(blocks, ws, winfs, P)
    Cs = [metrics(xy)[3] for xy in xys]
    nbr = [cut_ghost_centres(blocks, P, Cs, k) for k in range(len(blocks))]
    return wes, nbr


def residual_all(blocks, q, flow, solver, cuts=(), alpha0=None, xys=None) -> torch.Tensor:
    """R* of all blocks (concatenated public layout); `cuts` glue block sides
    (cut_partners), `xys`/`alpha0` override node coordinates / incidence."""
    xys = [b.xy for b in blocks] if xys is None else xys
    qs = split(blocks, q)
    wes, nbr = _halos(blocks, qs, flow, cuts, alpha0, xys)
    return join([residual(b, qb, flow, solver, alpha0, xy, we, nc)
                 for b, qb, xy, we, nc in zip(blocks, qs, xys, wes, nbr)])


# ---------------------------------------------------------------------------
# Local time step and Runge-Kutta
# ---------------------------------------------------------------------------
def local_dt(b: OBlock, q0: torch.Tensor, flow: OFlow, solver: OSolver) -> torch.Tensor:
    """Local pseudo-time step per cell and snapshot, from the iteration's
    starting state:  dtau = CFL V / (L_I + L_J + 4 (Lv_I + Lv_J) + V omega N_H),
    L_I = |u . S_I~| + c |S_I~| with S_I~ the mean of the cell's two i-face
    normals (same for J), Lv = max(4/(3 rho), gamma/rho) (mu/Pr) |S~|^2 / V.
    The last term bounds the spectral radius omega N_H of the HB operator."""
    g = flow.gamma
    SI, SJ, V, _ = metrics(b.xy)
    w = primitives(q0, g)
    rho, u, v, p = w[:, 0], w[:, 1], w[:, 2], w[:, 3]
    c = torch.sqrt(g * p / rho)
    si = 0.5 * (SI[:, :-1, :] + SI[:, 1:, :])
    sj = 0.5 * (SJ[:-1, :, :] + SJ[1:, :, :])
    ai = torch.sqrt(si[..., 0] ** 2 + si[..., 1] ** 2)
    aj = torch.sqrt(sj[..., 0] ** 2 + sj[..., 1] ** 2)
    li = torch.abs(u * si[..., 0] + v * si[..., 1]) + c * ai
    lj = torch.abs(u * sj[..., 0] + v * sj[..., 1]) + c * aj
    fac = torch.maximum(4.0 / (3.0 * rho), g / rho) * (flow.mu / flow.prandtl)
    lvi = fac * ai * ai / V
    lvj = fac * aj * aj / V
    lam = li + lj + 4.0 * (lvi + lvj) + V * flow.omega * b.n_harm
    return solver.cfl * V / lam


def rk_stages(q0, dt_over_v, resid, alphas):
    """One pseudo-time iteration of the low-storage multistage scheme:
    Q(k) = Q(0) - alpha_k (dtau/V) R*(Q(k-1)), k = 1..len(alphas).
    `resid` maps a state to R*; returns (Q(last), R*(Q(0)))."""
    qk = q0
    r0 = None
    for a in alphas:
        r = resid(qk)
        if r0 is None:
            r0 = r
        qk = q0 - a * dt_over_v * r
    return qk, r0


def rk_iterate(blocks, q: torch.Tensor, flow, solver, n_iter: int, cuts=()):
    """Explicit multistage Runge-Kutta pseudo-time iterations (the paper's
    "Runge-Kutta step", §MPI Optimisations; coefficients not given there).

    Reading: four-stage low-storage scheme
        Q(k) = Q(0) - alpha_k (dtau / V) R*(Q(k-1)),  alpha = (1/4, 1/3, 1/2, 1),
    every term re-evaluated at every stage, dtau from Q(0) and frozen over the
    stages.  Residual norm of iteration it: RMS over all blocks, cells and
    snapshots of R*_rho / V at the first stage.
    Returns (state after n_iter iterations, norms[n_iter])."""
    q = q.clone()
    norms = []
    total = sum(b.ns * b.ni * b.nj for b in blocks)
    vols = [metrics(b.xy)[2] for b in blocks]
    for _ in range(n_iter):
        q0 = split(blocks, q)
        dtv = join([(local_dt(b, qb, flow, solver) / V)[:, None].expand(-1, 4, -1, -1)
                    for b, qb, V in zip(blocks, q0, vols)])
        resid = lambda x: residual_all(blocks, x, flow, solver, cuts)
        q, r0 = rk_stages(q, dtv, resid, solver.rk_alpha)
        s = sum(float(((r[:, 0] / V) ** 2).sum())
                for r, V in zip(split(blocks, r0), vols))
        norms.append(math.sqrt(s / total))
    return q, torch.tensor(norms, dtype=DT)


def td_march(b: OBlock, q: torch.Tensor, flow: OFlow, solver: OSolver, dt: float,
             n_steps: int, t0: float = 0.0, alpha_amps: Optional[Sequence[float]] = None):
    """Time-domain reference: classical fourth-order Runge-Kutta in physical
    time on V dQ/dt = -R(Q, t) (no HB term), with the far field at the
    instantaneous incidence alpha(t) = alpha0 + A sin(omega t).  q is a
    single-snapshot state [1][4][nj][ni].  Returns the state at t0 + n dt.

    Independent marches of the same block may share the call: q[r] is then
    the state of march r, forced with amplitude alpha_amps[r] (the rows do
    not interact: the spatial operator treats each row on its own)."""
    V = metrics(b.xy)[2]
    amps = [flow.alpha_amp] * q.shape[0] if alpha_amps is None else list(alpha_amps)
    if len(amps) != q.shape[0]:
        raise ValueError("one forcing amplitude per state row")

    def f(x, t):
        rows = []
        for A in amps:
            a = flow.alpha0 + A * math.sin(flow.omega * t)
            rows.append([1.0, flow.mach * math.cos(a), flow.mach * math.sin(a),
                         1.0 / flow.gamma])
        winf = torch.tensor(rows, dtype=DT)
        return -spatial_residual(b, x, flow, solver, winf=winf) / V

    t = t0
    for _ in range(n_steps):
        k1 = f(q, t)
        k2 = f(q + 0.5 * dt * k1, t + 0.5 * dt)
        k3 = f(q + 0.5 * dt * k2, t + 0.5 * dt)
        k4 = f(q + dt * k3, t + dt)
        q = q + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        t += dt
    return q


# ---------------------------------------------------------------------------
# Forces
# ---------------------------------------------------------------------------
def wall_face_mask(b: OBlock, nbrC=None) -> torch.Tensor:
    """jmin faces that are solid wall (all of them for WALL, the profile part
    for WAKECUT, the cells no segment covers for CUT_WALL: `nbrC` as in
    ghost_centres).  Only jmin walls carry loads in these grids."""
    i = torch.arange(b.ni)
    if b.bc[2] == WALL:
        return torch.ones(b.ni, dtype=torch.bool)
    if b.bc[2] == WAKECUT:
        return (i >= b.wake_ncells) & (i < b.ni - b.wake_ncells)
    if b.bc[2] == CUT_WALL:
        return torch.isnan(nbrC[2][:, 0])
    return torch.zeros(b.ni, dtype=torch.bool)


def block_loads(b: OBlock, q: torch.Tensor, flow: OFlow,
                alpha0: Optional[torch.Tensor] = None, xy: Optional[torch.Tensor] = None,
                we: Optional[torch.Tensor] = None, nbrC=None):
    """Force (Fx, Fy) and moment Mz (counter-clockwise positive, about
    (x_mom, y_mom)) on the wall faces of one block, per snapshot, [ns][3].

    Per wall face (normal S_J pointing into the fluid): pressure part
    -(p_w - p_inf) S with p_w the adjacent interior cell's pressure; viscous
    part tau . S with tau from the wall-face diamond gradient (the same
    stress as in the residual).  The moment arm is the face midpoint."""
    g = flow.gamma
    xy = b.xy if xy is None else xy
    SI, SJ, V, C = metrics(xy)
    ns = q.shape[0]
    w = primitives(q, g)
    if we is None:
        we = extend(b, w, freestream_prim(flow, ns, alpha0))
    t = uvt(we, g)
    ni, nj = b.ni, b.nj
    nodev = 0.25 * (t[:, :, 1:3, 1:ni + 2] + t[:, :, 1:3, 2:ni + 3]
                    + t[:, :, 2:4, 1:ni + 2] + t[:, :, 2:4, 2:ni + 3])   # nodes j = 0, 1
    cjm = ghost_centres(b, xy, C, nbrC)[2]
    S = SJ[0].permute(1, 0)                          # [2][ni]
    tL = t[:, :, 1, 2:ni + 2]
    tR = t[:, :, 2, 2:ni + 2]
    nA = nodev[:, :, 0, 0:ni]
    nB = nodev[:, :, 0, 1:ni + 1]
    cL = cjm.permute(1, 0)
    cR = C[0].permute(1, 0)
    pA = xy[:, 0, 0:ni]
    pB = xy[:, 0, 1:ni + 1]
    G = viscous_face_flux(tL.transpose(0, 1), tR.transpose(0, 1), nB.transpose(0, 1),
                          nA.transpose(0, 1), cL, cR, pB, pA, S, flow)   # [4][ns][ni]
    pw = w[:, 3, 0, :]                               # [ns][ni]
    pinf = 1.0 / g
    fx = -(pw - pinf) * S[0] + G[1]
    fy = -(pw - pinf) * S[1] + G[2]
    mx = 0.5 * (pA[0] + pB[0]) - flow.x_mom
    my = 0.5 * (pA[1] + pB[1]) - flow.y_mom
    mz = mx * fy - my * fx
    m = wall_face_mask(b, nbrC).to(DT)
    return torch.stack([(fx * m).sum(-1), (fy * m).sum(-1), (mz * m).sum(-1)], dim=-1)


def forces(blocks, q: torch.Tensor, flow: OFlow, solver: OSolver,
           alpha0: Optional[torch.Tensor] = None, cuts=(), xys=None) -> List[torch.Tensor]:
    """Lift, drag and moment coefficients per body and snapshot (the paper's
    cl(n, ibody), cd(n, ibody), cm(n, ibody), §MPI Optimisations, force
    reduction).  Axes of the mean free stream: drag along (cos a0, sin a0),
    lift along (-sin a0, cos a0); coefficients on q_inf = M^2/2 and the unit
    reference length; cm positive nose-up (clockwise), i.e. -Mz/(q_inf L^2).
    Returns a list over bodies of [ns][3] = (cl, cd, cm)."""
    a0 = flow.alpha0 if alpha0 is None else alpha0
    a0 = torch.as_tensor(a0, dtype=DT)
    qinf = 0.5 * flow.mach ** 2
    nbody = max(b.body_id for b in blocks) + 1
    acc = [None] * nbody
    xys = [b.xy for b in blocks] if xys is None else xys
    qs = split(blocks, q)
    wes, nbr = _halos(blocks, qs, flow, cuts, alpha0, xys)
    for b, qb, xy, we, nc in zip(blocks, qs, xys, wes, nbr):
        L = block_loads(b, qb, flow, alpha0, xy, we, nc)
        acc[b.body_id] = L if acc[b.body_id] is None else acc[b.body_id] + L
    out = []
    for L in acc:
        fx, fy, mz = L[:, 0], L[:, 1], L[:, 2]
        cd = (fx * torch.cos(a0) + fy * torch.sin(a0)) / (qinf * flow.l_ref)
        cl = (-fx * torch.sin(a0) + fy * torch.cos(a0)) / (qinf * flow.l_ref)
        cm = -mz / (qinf * flow.l_ref ** 2)
        out.append(torch.stack([cl, cd, cm], dim=-1))
    return out


def harmonics(c: torch.Tensor) -> torch.Tensor:
    """Fourier coefficients of a snapshot series c[ns] (real DFT):
    returns [a0, a1, b1, ..., aN, bN] with c(t) = a0 + sum a_k cos + b_k sin."""
    ns = c.shape[0]
    nh = (ns - 1) // 2
    n = torch.arange(ns, dtype=DT)
    out = [c.mean()]
    for k in range(1, nh + 1):
        out.append(2.0 / ns * (c * torch.cos(2 * math.pi * k * n / ns)).sum())
        out.append(2.0 / ns * (c * torch.sin(2 * math.pi * k * n / ns)).sum())
    return torch.stack(out)


# ---------------------------------------------------------------------------
# Reverse mode (for checking the adjoint)
# ---------------------------------------------------------------------------
def residual_vjp(blocks, q: torch.Tensor, flow: OFlow, solver: OSolver, rbar: torch.Tensor,
                 cuts=()):
    """Products of the transposed Jacobians of R* (all blocks) with rbar, by
    automatic differentiation of this module's residual: returns
    (qbar, [xybar per block], alpha0bar).  Pinned against central finite
    differences in the tests."""
    qv = q.detach().clone().requires_grad_(True)
    xys = [b.xy.detach().clone().requires_grad_(True) for b in blocks]
    a0 = torch.tensor(flow.alpha0, dtype=DT, requires_grad=True)
    (residual_all(blocks, qv, flow, solver, cuts, a0, xys) * rbar).sum().backward()
    return qv.grad.detach(), [x.grad.detach() for x in xys], a0.grad.detach()


def forces_vjp(blocks, q: torch.Tensor, flow: OFlow, solver: OSolver, cfbar: torch.Tensor,
               cuts=()):
    """Products of the transposed Jacobians of the force coefficients (all
    bodies, [body][n][3] flattened) with cfbar, by automatic differentiation
    of forces(): returns (qbar, [xybar per block], alpha0bar)."""
    qv = q.detach().clone().requires_grad_(True)
    xys = [b.xy.detach().clone().requires_grad_(True) for b in blocks]
    a0 = torch.tensor(flow.alpha0, dtype=DT, requires_grad=True)
    cf = torch.cat([c.reshape(-1) for c in forces(blocks, qv, flow, solver, a0, cuts, xys)])
    (cf * cfbar).sum().backward()
    return qv.grad.detach(), [x.grad.detach() for x in xys], a0.grad.detach()


def forces_with(blocks, q, flow, solver, xys=None, alpha0=None, cuts=()):
    """Force coefficients (flattened [body][n][3]) with node coordinates
    and/or alpha0 overridden."""
    a0 = None if alpha0 is None else torch.as_tensor(alpha0, dtype=DT)
    return torch.cat([c.reshape(-1) for c in forces(blocks, q, flow, solver, a0, cuts, xys)])


def residual_with(blocks, q, flow, solver, xys=None, alpha0=None, cuts=()):
    """R* of all blocks with node coordinates and/or alpha0 overridden."""
    a0 = None if alpha0 is None else torch.as_tensor(alpha0, dtype=DT)
    return residual_all(blocks, q, flow, solver, cuts, a0, xys)
