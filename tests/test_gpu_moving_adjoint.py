"""Adjoint kernels on a rigidly heaving and pitching grid (hb_set_motion):
the transposed-Jacobian products of the moving-grid R* and force
coefficients with respect to the state, the body-frame node coordinates
(through the rotated face vectors, the face speeds, the moving-wall images
and the moment arm) and the mean incidence against the FP64 moving-grid
oracle's reverse mode (element by element), the adjoint pseudo-time
iteration stage by stage against the oracle's products and moving-grid
local steps, and dot-product checks against central differences of the
GPU's own moving-grid residual in the state and in the nodes."""
import sys

import pytest
import torch

from oracle import hb_moving as M
from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
MOT = dict(pitch_amp=0.3, pitch_phase=0.5, heave_amp=1.5, x_pivot=0.25, y_pivot=0.05)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float((a - b).norm() / b.norm())


def _case(name, pi, pj):
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.02
    q = torch.as_tensor(synth.initial_state(p))
    if pi * pj > 1:
        p, perm = synth.split_problem(p, pi, pj)
        q = q[torch.as_tensor(perm)].contiguous()
    blocks, flow, solver = O.from_synth(p)
    return p, blocks, flow, solver, q


def _grid(p, batched):
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=0, batched=batched)
    g.set_motion(**MOT)
    return g


CASES = [("cyl_tiny", 1, 1, 0), ("cyl_tiny", 1, 1, 1), ("naca_tiny", 1, 1, 0),
         ("naca_tiny", 1, 1, 1), ("batch_tiny", 1, 1, 1), ("cyl_tiny", 2, 2, 1), ("naca_tiny", 1, 2, 0)]
IDS = ["cyl-plain", "cyl-batched", "naca-plain", "naca-batched", "batch", "cyl2x2", "naca1x2-plain"]


@pytest.mark.parametrize("name,pi,pj,batched", CASES, ids=IDS)
def test_moving_residual_adjoint_matches_oracle(name, pi, pj, batched):
    _say("moving residual adjoint", name, pi, pj, "batched", batched)
    p, blocks, flow, solver, q = _case(name, pi, pj)
    m = M.OMotion(**MOT)
    rbar = torch.randn(q.shape, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    qref, xref, aref = M.moving_residual_vjp(blocks, q, flow, solver, m, rbar, p.cuts)
    qfix = O.residual_vjp(blocks, q, flow, solver, rbar, p.cuts)[0]
    assert _rel(qfix, qref) > 1e-3                     # the motion matters
    g = _grid(p, batched)
    qb = torch.empty_like(q, device=DEV)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    g.residual_adjoint(q.to(DEV), rbar.to(DEV), qb, xyb, ab)
    torch.cuda.synchronize()
    qb = qb.cpu()
    xr = torch.cat([x.reshape(-1) for x in xref])
    _say("  qbar rel", _rel(qb, qref), "xybar rel", _rel(xyb.cpu(), xr), "alpha", float(ab), float(aref))
    assert _rel(qb, qref) <= 1e-11
    assert float((qb - qref).abs().max()) <= 1e-10 * float(qref.abs().max())
    assert _rel(xyb.cpu(), xr) <= 1e-11
    assert abs(float(ab) - float(aref)) <= 1e-11 * abs(float(aref))
    # without coordinates: the same qbar up to rounding (the face kernel
    # that skips the coordinate records is compiled separately, and its
    # shared arithmetic may fuse multiply-adds differently)
    qb2 = g.residual_adjoint(q.to(DEV), rbar.to(DEV))
    torch.cuda.synchronize()
    _say("  qbar without coordinates: rel to qbar", _rel(qb2.cpu(), qb))
    assert _rel(qb2.cpu(), qb) <= 1e-13
    assert _rel(qb2.cpu(), qref) <= 1e-11
    g.close()


@pytest.mark.parametrize("name,pi,pj,batched", [CASES[1], CASES[3], CASES[5]], ids=[IDS[1], IDS[3], IDS[5]])
def test_moving_forces_adjoint_matches_oracle(name, pi, pj, batched):
    _say("moving forces adjoint", name, pi, pj, "batched", batched)
    p, blocks, flow, solver, q = _case(name, pi, pj)
    m = M.OMotion(**MOT)
    g = _grid(p, batched)
    cfbar = torch.randn(g.n_forces, generator=torch.Generator().manual_seed(5), dtype=torch.float64)
    qref, xref, aref = M.moving_forces_vjp(blocks, q, flow, solver, m, cfbar, p.cuts)
    qb = torch.empty_like(q, device=DEV)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    g.forces_adjoint(q.to(DEV), cfbar.to(DEV), qb, xyb, ab)
    torch.cuda.synchronize()
    qb = qb.cpu()
    xr = torch.cat([x.reshape(-1) for x in xref])
    _say("  qbar rel", _rel(qb, qref), "xybar rel", _rel(xyb.cpu(), xr), "alpha", float(ab), float(aref))
    assert _rel(qb, qref) <= 1e-11
    assert _rel(xyb.cpu(), xr) <= 1e-11
    assert abs(float(ab) - float(aref)) <= 1e-11 * abs(float(aref))
    g.close()


def test_moving_adjoint_iteration_stage_by_stage():
    """Two adjoint iterations lam <- lam0 - alpha_k (dtau/V)(J^T lam + gq)
    with the moving grid's local steps, against the same recursion on the
    oracle's reverse products; the first-stage norms too."""
    p, blocks, flow, solver, q = _case("cyl_tiny", 1, 1)
    m = M.OMotion(**MOT)
    gen = torch.Generator().manual_seed(8)
    gq = torch.randn(q.shape, generator=gen, dtype=torch.float64)
    lam = 1e-2 * torch.randn(q.shape, generator=gen, dtype=torch.float64)
    g = _grid(p, 1)
    lg = lam.to(DEV)
    norms = torch.zeros(2, dtype=torch.float64, device=DEV)
    g.adjoint_iterate(q.to(DEV), lg, gq.to(DEV), 2, norms)
    torch.cuda.synchronize()
    vols = [O.metrics(b.xy)[2] for b in blocks]
    dtv = O.join([(M.moving_local_dt(b, qb, flow, solver, m) / V)[:, None].expand(-1, 4, -1, -1)
                  for b, qb, V in zip(blocks, O.split(blocks, q), vols)])
    ref_norms = []
    for _ in range(2):
        lam0 = lam.clone()
        for k, a in enumerate(solver.rk_alpha):
            r = M.moving_residual_vjp(blocks, q, flow, solver, m, lam, p.cuts)[0] + gq
            if k == 0:
                s = sum(float(((rb / V) ** 2).sum()) for rb, V in zip(O.split(blocks, r), vols))
                ref_norms.append((s / q.numel()) ** 0.5)
            lam = lam0 - a * dtv * r
    err = _rel(lg.cpu(), lam)
    _say("  lambda rel", err, "norms", norms.cpu().tolist(), ref_norms)
    assert err <= 1e-11
    for a, b in zip(norms.cpu().tolist(), ref_norms):
        assert abs(a - b) <= 1e-11 * b
    g.close()


def test_moving_adjoint_dot_product_with_gpu_differences():
    """<rbar, (R(q+hv) - R(q-hv)) / 2h> = <J^T rbar, v> on the moving grid,
    using only the GPU."""
    p, blocks, flow, solver, q = _case("naca_tiny", 1, 1)
    q = q.to(DEV)
    gen = torch.Generator().manual_seed(11)
    rbar = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV)
    v = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV) * q.abs() * 1e-2
    g = _grid(p, 1)
    qb = g.residual_adjoint(q, rbar)
    h = 1e-6
    fd = float((rbar * (g.residual(q + h * v) - g.residual(q - h * v))).sum()) / (2 * h)
    ad = float((qb * v).sum())
    _say("  fd", fd, "adjoint", ad)
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    g.close()


def test_moving_coordinate_adjoint_dot_product_with_gpu_differences():
    """<rbar, (R(x+hv) - R(x-hv)) / 2h> = <xybar, v> for the body-frame node
    coordinates on the moving grid (hb_set_xy moves the body-frame grid),
    using only the GPU."""
    p, blocks, flow, solver, q = _case("naca_tiny", 1, 1)
    q = q.to(DEV)
    gen = torch.Generator().manual_seed(12)
    rbar = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV)
    g = _grid(p, 1)
    xy0 = torch.as_tensor(p.blocks[0].xy.reshape(-1)).to(DEV)
    v = torch.randn(xy0.shape, generator=gen, dtype=torch.float64).to(DEV) * 1e-3
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    g.residual_adjoint(q, rbar, None, xyb)
    h = 1e-6

    def r_at(xy):
        g.set_xy(xy)
        return g.residual(q)

    fd = float((rbar * (r_at(xy0 + h * v) - r_at(xy0 - h * v))).sum()) / (2 * h)
    ad = float((xyb * v).sum())
    _say("  fd", fd, "adjoint", ad)
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    g.close()
