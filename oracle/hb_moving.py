"""FP64 CPU oracle of the HB residual, pseudo-time iteration and loads on a
rigidly heaving and pitching grid (the paper's test case 1 is a heaving and
pitching wing, §Experimental Setup, Test case 1; the paper gives no moving-
grid equations).

TEST INFRASTRUCTURE ONLY, like hb_oracle (same import rules; it shares no
code with the HIP library).

Reading (the textbook arbitrary Lagrangian-Eulerian finite-volume form):
  * the whole grid moves rigidly.  Snapshot n (omega t_n = 2 pi n / N_s)
    holds the body-frame nodes x0 rotated counter-clockwise by theta_n about
    the pivot p and raised by h_n:  x_n = R(theta_n)(x0 - p) + p + (0, h_n),
    theta(t) = A_theta sin(omega t + phi), h(t) = A_h sin(omega t);
  * a grid point moves with the rigid velocity
    x_t = theta_dot k x (x - p - (0, h)) + (0, h_dot);
  * face flux F.S - (x_t . S) U with x_t at the face midpoint, Roe's
    dissipation on the eigenvalues relative to the face (roe_flux with vg);
    the viscous flux is the fixed-grid one on the snapshot's grid;
  * cell areas do not change, so the HB term stays V (D Q)_n, and the
    midpoint face speeds of a linear velocity field sum to zero around every
    cell (the discrete geometric conservation law holds exactly);
  * no-slip walls move: a wall ghost mirrors the velocity about the wall
    velocity, u_g = 2 u_w - u, u_w = x_t at the midpoint of the wall face
    of the mirrored cell's column (for corner ghosts: the i-periodic partner
    column, the glued block's column across an i cut, else the nearest
    column); cut ghosts are the glued block's cells of the same snapshot;
  * far field: the free stream at the (fixed) incidence alpha0 (plus any
    alpha_amp forcing, unchanged);
  * local time step: the fixed-grid formula on the snapshot's grid with the
    velocity relative to the grid at the cell centre;
  * loads: fixed-grid loads on the snapshot's grid, the moment about the
    reference point carried with the body; lift and drag along the mean
    free stream.
Grids with i-side walls are outside this reading (ValueError).

Parity status: pinned in tests/test_oracle_moving.py (zero motion, heave as
a Galilean shift, rotation equivariance, free-stream preservation on a
pitching and heaving grid, grid velocity against differenced positions,
no-slip wall images, a block cut into glued pieces, the time-domain march at
zero motion).  Converged N_H = 1 snapshots against the moving-grid
time-domain march are compared on the GPU (tests/test_gpu_moving.py).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import List, Sequence

import torch

from oracle import hb_oracle as O

DT = torch.float64


@dataclass
class OMotion:
    pitch_amp: float = 0.0      # A_theta, radians, counter-clockwise positive
    pitch_phase: float = 0.0    # phi, radians (pitch leads heave by phi)
    heave_amp: float = 0.0      # A_h, in the length unit of the grid, +y
    x_pivot: float = 0.0
    y_pivot: float = 0.0


def motion_at(m: OMotion, omega: float, phase: float):
    """(theta, theta_dot, h, h_dot) at omega t = phase."""
    th = m.pitch_amp * math.sin(phase + m.pitch_phase)
    thd = omega * m.pitch_amp * math.cos(phase + m.pitch_phase)
    h = m.heave_amp * math.sin(phase)
    hd = omega * m.heave_amp * math.cos(phase)
    return th, thd, h, hd


def snapshot_motion(m: OMotion, flow: O.OFlow, ns: int, n: int):
    return motion_at(m, flow.omega, 2.0 * math.pi * n / ns)


def place(m: OMotion, th: float, h: float, x: torch.Tensor, y: torch.Tensor):
    """Body-frame points (x, y) after the rotation by th about the pivot and
    the rise h."""
    c, s = math.cos(th), math.sin(th)
    dx, dy = x - m.x_pivot, y - m.y_pivot
    return m.x_pivot + c * dx - s * dy, m.y_pivot + h + s * dx + c * dy


def rigid_velocity(m: OMotion, thd: float, h: float, hd: float, x: torch.Tensor,
                   y: torch.Tensor):
    """Velocity of the grid point that is now at (x, y)."""
    rx, ry = x - m.x_pivot, y - (m.y_pivot + h)
    return -thd * ry, thd * rx + hd


def snapshot_xy(b: O.OBlock, m: OMotion, flow: O.OFlow, n: int) -> torch.Tensor:
    th, _, h, _ = snapshot_motion(m, flow, b.ns, n)
    x, y = place(m, th, h, b.xy[0], b.xy[1])
    return torch.stack([x, y])


def face_speeds(xy: torch.Tensor, m: OMotion, thd: float, h: float, hd: float):
    """x_t . S of every i-face [nj][ni+1] and j-face [nj+1][ni] of a grid
    (x_t at the face midpoint)."""
    SI, SJ, _, _ = O.metrics(xy)
    x, y = xy[0], xy[1]
    ux, uy = rigid_velocity(m, thd, h, hd, 0.5 * (x[:-1, :] + x[1:, :]), 0.5 * (y[:-1, :] + y[1:, :]))
    vgi = ux * SI[..., 0] + uy * SI[..., 1]
    ux, uy = rigid_velocity(m, thd, h, hd, 0.5 * (x[:, :-1] + x[:, 1:]), 0.5 * (y[:, :-1] + y[:, 1:]))
    vgj = ux * SJ[..., 0] + uy * SJ[..., 1]
    return vgi, vgj


def check_block(b: O.OBlock):
    if any(b.bc[s] in (O.WALL, O.CUT_WALL) for s in (0, 1)):
        raise ValueError("moving grids: walls only on j sides")


def wall_images(blocks, cutmap: dict, k: int, we: torch.Tensor, xys, m: OMotion, thd: float,
                h: float, hd: float):
    """Add 2 u_w to the velocity of the no-slip wall images of block k's
    extended field we (in place; the fixed-grid rule gave -u): u_w = the grid
    velocity at the midpoint of the wall face at which the ghost's
    resolution mirrored (hb_oracle.wall_map; for a corner ghost that is the
    column its i-side rule led to: the i-periodic partner column, or the
    glued block's column across an i cut), on the moved nodes xys of the
    block holding that face."""
    walls = O.wall_map(blocks, cutmap, k)
    if not walls:
        return we
    if any(w[3] < 2 for w in walls):
        raise ValueError("moving grids: walls only on j sides")
    for wb in sorted(set(w[2] for w in walls)):
        sel = [w for w in walls if w[2] == wb]
        xy = xys[wb]
        je = torch.tensor([w[0] for w in sel])
        ie = torch.tensor([w[1] for w in sel])
        jw = torch.tensor([0 if w[3] == 2 else xy.shape[-2] - 1 for w in sel])
        pos = torch.tensor([w[4] for w in sel])
        ux, uy = rigid_velocity(m, thd, h, hd, 0.5 * (xy[0, jw, pos] + xy[0, jw, pos + 1]),
                                0.5 * (xy[1, jw, pos] + xy[1, jw, pos + 1]))
        we[:, 1, je, ie] += 2.0 * ux
        we[:, 2, je, ie] += 2.0 * uy
    return we


def moving_extend(b: O.OBlock, w: torch.Tensor, winf: torch.Tensor, xy: torch.Tensor,
                  m: OMotion, thd: float, h: float, hd: float) -> torch.Tensor:
    """Ghost-extended primitives of one snapshot (w[1][4][nj][ni], winf[1][4])
    of a block without cuts on the moved grid xy: the fixed-grid rules
    (hb_oracle.extend), then the moving-wall images  u_g = 2 u_w - u."""
    check_block(b)
    if any(k in O.GLUED for k in b.bc):
        raise ValueError("moving_extend: a block with cuts needs its neighbours (moving_snapshots)")
    return wall_images([b], {}, 0, O.extend(b, w, winf).clone(), [xy], m, thd, h, hd)


def moving_snapshots(blocks: Sequence[O.OBlock], qs, flow: O.OFlow, m: OMotion, cuts=(),
                     alpha0=None, body_xys=None):
    """For every block k and snapshot n: (k, n, moved nodes, ghost-extended
    primitives with moving-wall images, moved centres of the glued blocks,
    (theta, theta_dot, h, h_dot)).  Cut ghosts are the glued block's cells of
    the same snapshot (hb_oracle.extend_all); glued blocks share N_s.
    `alpha0` (a 0-d tensor) overrides the mean incidence of the far field,
    `body_xys` the body-frame nodes of the blocks."""
    P = O.cut_partners(blocks, cuts) if cuts else {}
    for b in blocks:
        check_block(b)
    ws = [O.primitives(qb, flow.gamma) for qb in qs]
    winfs = [O.freestream_prim(flow, b.ns, alpha0) for b in blocks]
    for n in range(max(b.ns for b in blocks)):
        # a block with fewer snapshots stands in with its last one; no block
        # glued to it reads that (glued blocks share N_s)
        sel = [min(n, b.ns - 1) for b in blocks]
        wes = O.extend_all(blocks, [w[s:s + 1] for w, s in zip(ws, sel)],
                           [f[s:s + 1] for f, s in zip(winfs, sel)], P)
        mot = [snapshot_motion(m, flow, b.ns, s) for b, s in zip(blocks, sel)]
        bxy = [b.xy for b in blocks] if body_xys is None else body_xys
        xys = [torch.stack(place(m, mt[0], mt[2], x[0], x[1])) for x, mt in zip(bxy, mot)]
        for k, b in enumerate(blocks):
            if n >= b.ns:
                continue
            _, thd, h, hd = mot[k]
            we = wall_images(blocks, P, k, wes[k].clone(), xys, m, thd, h, hd)
            Cs = [O.metrics(xy)[3] for xy in xys]
            nbrC = O.cut_ghost_centres(blocks, P, Cs, k) or None
            yield k, n, xys[k], we, nbrC, mot[k]


def _snapshot(b, w, winf, m, flow, n):
    th, thd, h, hd = snapshot_motion(m, flow, b.ns, n)
    xy = snapshot_xy(b, m, flow, n)
    we = moving_extend(b, w[n:n + 1], winf[n:n + 1], xy, m, thd, h, hd)
    return xy, we, (th, thd, h, hd)


def moving_flux_balance(b: O.OBlock, q1: torch.Tensor, flow: O.OFlow, solver: O.OSolver,
                        m: OMotion, phase: float, winf1: torch.Tensor) -> torch.Tensor:
    """Net moving-face outflow of each cell for a one-snapshot state
    q1[1][4][nj][ni] on the grid at omega t = phase, far field winf1[1][4]."""
    th, thd, h, hd = motion_at(m, flow.omega, phase)
    xy = torch.stack(place(m, th, h, b.xy[0], b.xy[1]))
    we = moving_extend(b, O.primitives(q1, flow.gamma), winf1, xy, m, thd, h, hd)
    vg = face_speeds(xy, m, thd, h, hd)
    FI, FJ = O.face_fluxes(b, q1, flow, solver, xy=xy, we=we, vg=vg)
    return (FI[..., :, 1:] - FI[..., :, :-1]) + (FJ[..., 1:, :] - FJ[..., :-1, :])


def moving_residual(b: O.OBlock, q: torch.Tensor, flow: O.OFlow, solver: O.OSolver,
                    m: OMotion) -> torch.Tensor:
    """R*_n = sum over faces of the moving-face fluxes on grid n + V (D Q)_n."""
    winf = O.freestream_prim(flow, b.ns)
    parts = [moving_flux_balance(b, q[n:n + 1], flow, solver, m, 2.0 * math.pi * n / b.ns,
                                 winf[n:n + 1]) for n in range(b.ns)]
    return torch.cat(parts) + O.hb_source(b, q, flow)


def moving_td_march(b: O.OBlock, q: torch.Tensor, flow: O.OFlow, solver: O.OSolver, m: OMotion,
                    dt: float, n_steps: int, t0: float = 0.0) -> torch.Tensor:
    """Time-domain reference on the moving grid: hb_oracle.td_march (classical
    fourth-order Runge-Kutta in physical time on V dQ/dt = -R(Q, t)) with R
    the moving-face flux balance on the grid of time t (the cell areas do not
    change under the rigid motion).  q is a single-snapshot state."""
    V = O.metrics(b.xy)[2]

    def f(x, t):
        a = flow.alpha0 + flow.alpha_amp * math.sin(flow.omega * t)
        winf = torch.tensor([[1.0, flow.mach * math.cos(a), flow.mach * math.sin(a),
                              1.0 / flow.gamma]], dtype=DT)
        return -moving_flux_balance(b, x, flow, solver, m, flow.omega * t, winf) / V

    t = t0
    for _ in range(n_steps):
        k1 = f(q, t)
        k2 = f(q + 0.5 * dt * k1, t + 0.5 * dt)
        k3 = f(q + 0.5 * dt * k2, t + 0.5 * dt)
        k4 = f(q + dt * k3, t + dt)
        q = q + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        t += dt
    return q


def moving_residual_all(blocks: Sequence[O.OBlock], q: torch.Tensor, flow, solver,
                        m: OMotion, cuts=(), alpha0=None, body_xys=None) -> torch.Tensor:
    """R* of all blocks on the moving grid; `cuts` glue block sides;
    `alpha0` (a 0-d tensor) overrides the mean incidence, `body_xys` the
    body-frame nodes."""
    qs = O.split(blocks, q)
    parts = [[None] * b.ns for b in blocks]
    bxy = [b.xy for b in blocks] if body_xys is None else body_xys
    for k, n, xy, we, nbrC, (_, thd, h, hd) in moving_snapshots(blocks, qs, flow, m, cuts, alpha0,
                                                                 body_xys):
        vg = face_speeds(xy, m, thd, h, hd)
        FI, FJ = O.face_fluxes(blocks[k], qs[k][n:n + 1], flow, solver, xy=xy, we=we, vg=vg,
                               nbrC=nbrC)
        parts[k][n] = (FI[..., :, 1:] - FI[..., :, :-1]) + (FJ[..., 1:, :] - FJ[..., :-1, :])
    return O.join([torch.cat(p) + O.hb_source(b, qb, flow, x)
                   for p, b, qb, x in zip(parts, blocks, qs, bxy)])


def moving_local_dt(b: O.OBlock, q0: torch.Tensor, flow: O.OFlow, solver: O.OSolver,
                    m: OMotion) -> torch.Tensor:
    """hb_oracle.local_dt on snapshot n's grid with u - x_t(centre) in the
    convective spectral radii."""
    g = flow.gamma
    w = O.primitives(q0, g)
    out = []
    for n in range(b.ns):
        _, thd, h, hd = snapshot_motion(m, flow, b.ns, n)
        SI, SJ, V, C = O.metrics(snapshot_xy(b, m, flow, n))
        gx, gy = rigid_velocity(m, thd, h, hd, C[..., 0], C[..., 1])
        rho, u, v, p = w[n, 0], w[n, 1] - gx, w[n, 2] - gy, w[n, 3]
        c = torch.sqrt(g * p / rho)
        si = 0.5 * (SI[:, :-1, :] + SI[:, 1:, :])
        sj = 0.5 * (SJ[:-1, :, :] + SJ[1:, :, :])
        ai = torch.sqrt(si[..., 0] ** 2 + si[..., 1] ** 2)
        aj = torch.sqrt(sj[..., 0] ** 2 + sj[..., 1] ** 2)
        li = torch.abs(u * si[..., 0] + v * si[..., 1]) + c * ai
        lj = torch.abs(u * sj[..., 0] + v * sj[..., 1]) + c * aj
        fac = torch.maximum(4.0 / (3.0 * rho), g / rho) * (flow.mu / flow.prandtl)
        lam = li + lj + 4.0 * (fac * ai * ai / V + fac * aj * aj / V) + V * flow.omega * b.n_harm
        out.append(solver.cfl * V / lam)
    return torch.stack(out)


def moving_rk_iterate(blocks, q: torch.Tensor, flow, solver, m: OMotion, n_iter: int, cuts=()):
    """hb_oracle.rk_iterate with the moving-grid residual and time step."""
    q = q.clone()
    norms = []
    total = sum(b.ns * b.ni * b.nj for b in blocks)
    vols = [O.metrics(b.xy)[2] for b in blocks]
    for _ in range(n_iter):
        q0 = O.split(blocks, q)
        dtv = O.join([(moving_local_dt(b, qb, flow, solver, m) / V)[:, None].expand(-1, 4, -1, -1)
                      for b, qb, V in zip(blocks, q0, vols)])
        resid = lambda x: moving_residual_all(blocks, x, flow, solver, m, cuts)
        q, r0 = O.rk_stages(q, dtv, resid, solver.rk_alpha)
        s = sum(float(((r[:, 0] / V) ** 2).sum()) for r, V in zip(O.split(blocks, r0), vols))
        norms.append(math.sqrt(s / total))
    return q, torch.tensor(norms, dtype=DT)


def moving_forces(blocks, q: torch.Tensor, flow: O.OFlow, solver: O.OSolver,
                  m: OMotion, cuts=(), alpha0=None, body_xys=None) -> List[torch.Tensor]:
    """hb_oracle.forces on the moved grids: per snapshot the wall loads of
    grid n (moving-wall ghosts), the moment about the moved reference point,
    lift and drag along the mean free stream.  [body][ns][3] = (cl, cd, cm).
    `alpha0` (a 0-d tensor) overrides the mean incidence, `body_xys` the
    body-frame nodes."""
    a0 = torch.as_tensor(flow.alpha0 if alpha0 is None else alpha0, dtype=DT)
    qinf = 0.5 * flow.mach ** 2
    nbody = max(b.body_id for b in blocks) + 1
    acc = [None] * nbody
    qs = O.split(blocks, q)
    rows = [[None] * b.ns for b in blocks]
    for k, n, xy, we, nbrC, (th, _, h, _) in moving_snapshots(blocks, qs, flow, m, cuts, alpha0,
                                                              body_xys):
        xm, ym = place(m, th, h, torch.tensor(flow.x_mom, dtype=DT), torch.tensor(flow.y_mom, dtype=DT))
        fn = dataclasses.replace(flow, x_mom=float(xm), y_mom=float(ym))
        rows[k][n] = O.block_loads(blocks[k], qs[k][n:n + 1], fn, xy=xy, we=we, nbrC=nbrC)[0]
    for b, r in zip(blocks, rows):
        L = torch.stack(r)
        acc[b.body_id] = L if acc[b.body_id] is None else acc[b.body_id] + L
    out = []
    for L in acc:
        fx, fy, mz = L[:, 0], L[:, 1], L[:, 2]
        cd = (fx * torch.cos(a0) + fy * torch.sin(a0)) / (qinf * flow.l_ref)
        cl = (-fx * torch.sin(a0) + fy * torch.cos(a0)) / (qinf * flow.l_ref)
        cm = -mz / (qinf * flow.l_ref ** 2)
        out.append(torch.stack([cl, cd, cm], dim=-1))
    return out


# ---------------------------------------------------------------------------
# Reverse mode on the moving grid (for checking the adjoint)
# ---------------------------------------------------------------------------
def moving_residual_vjp(blocks, q: torch.Tensor, flow, solver, m: OMotion, rbar: torch.Tensor,
                        cuts=()):
    """Products of the transposed Jacobians of the moving-grid R* with rbar,
    by automatic differentiation of moving_residual_all: (qbar, [body-frame
    node bars per block], alpha0bar), the motion held fixed."""
    qv = q.detach().clone().requires_grad_(True)
    xys = [b.xy.detach().clone().requires_grad_(True) for b in blocks]
    a0 = torch.tensor(flow.alpha0, dtype=DT, requires_grad=True)
    (moving_residual_all(blocks, qv, flow, solver, m, cuts, a0, xys) * rbar).sum().backward()
    return qv.grad.detach(), [x.grad.detach() for x in xys], a0.grad.detach()


def moving_forces_vjp(blocks, q: torch.Tensor, flow, solver, m: OMotion, cfbar: torch.Tensor,
                      cuts=()):
    """Products of the transposed Jacobians of the moving-grid force
    coefficients (flattened [body][n][3]) with cfbar: (qbar, [body-frame
    node bars per block], alpha0bar)."""
    qv = q.detach().clone().requires_grad_(True)
    xys = [b.xy.detach().clone().requires_grad_(True) for b in blocks]
    a0 = torch.tensor(flow.alpha0, dtype=DT, requires_grad=True)
    cf = torch.cat([c.reshape(-1) for c in moving_forces(blocks, qv, flow, solver, m, cuts, a0, xys)])
    (cf * cfbar).sum().backward()
    return qv.grad.detach(), [x.grad.detach() for x in xys], a0.grad.detach()
