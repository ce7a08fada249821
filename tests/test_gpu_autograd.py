"""GPU parity of the forces adjoint and of the torch.autograd wrappers:
hb_forces_adjoint against the FP64 oracle's reverse mode of its force
coefficients, and gradients through autograd.residual / autograd.forces
against the oracle's reverse mode of the same objective."""
import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import autograd as A
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("name", ["cyl_tiny", "naca_tiny", "batch_tiny"])
@pytest.mark.parametrize("prec,batched", [(0, 0), (0, 1), (1, 1)])
def test_forces_adjoint_matches_oracle(name, prec, batched):
    _say("forces adjoint", name, prec, batched)
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.02
    blocks, flow, solver = O.from_synth(p)
    q = torch.as_tensor(synth.initial_state(p))
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=prec, batched=batched)
    cfbar = torch.randn(g.n_forces, generator=torch.Generator().manual_seed(2), dtype=torch.float64)
    qref, xref, aref = O.forces_vjp(blocks, q, flow, solver, cfbar)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    qb = g.forces_adjoint(q.to(DEV), cfbar.to(DEV), None, xyb, ab)
    torch.cuda.synchronize()
    xr = torch.cat([x.reshape(-1) for x in xref])
    _say("  qbar", _rel(qb.cpu(), qref), "xybar", _rel(xyb.cpu(), xr), "alpha", float(ab), float(aref))
    assert _rel(qb.cpu(), qref) <= 1e-11
    assert _rel(xyb.cpu(), xr) <= 1e-11
    assert abs(float(ab) - float(aref)) <= 1e-11 * abs(float(aref))


def test_forces_adjoint_split_grid():
    p = synth.make_problem("cyl_tiny")
    sp, perm = synth.split_problem(p, 2, 2)
    sblocks, flow, solver = O.from_synth(sp)
    q = torch.as_tensor(synth.initial_state(p))[torch.as_tensor(perm)].contiguous()
    g = hb.Grid(sp.blocks, sp.flow, sp.solver, cuts=sp.cuts, precision=0, batched=1)
    cfbar = torch.randn(g.n_forces, generator=torch.Generator().manual_seed(6), dtype=torch.float64)
    qref, xref, aref = O.forces_vjp(sblocks, q, flow, solver, cfbar, sp.cuts)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    qb = g.forces_adjoint(q.to(DEV), cfbar.to(DEV), None, xyb, ab)
    torch.cuda.synchronize()
    assert _rel(qb.cpu(), qref) <= 1e-11
    assert _rel(xyb.cpu(), torch.cat([x.reshape(-1) for x in xref])) <= 1e-11


def test_autograd_residual_and_forces():
    """loss = <w, R*(q; X, a0)> + <c, cf(q; X, a0)> through the autograd
    wrappers; gradients of q, X and a0 against the oracle's reverse mode."""
    p = synth.make_problem("naca_tiny")
    blocks, flow, solver = O.from_synth(p)
    q0 = torch.as_tensor(synth.initial_state(p))
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    gen = torch.Generator().manual_seed(21)
    w = torch.randn(q0.shape, generator=gen, dtype=torch.float64)
    c = torch.randn(g.n_forces, generator=gen, dtype=torch.float64)
    q = q0.to(DEV).requires_grad_(True)
    xy = torch.as_tensor(p.blocks[0].xy).reshape(-1).to(DEV).requires_grad_(True)
    a0 = torch.tensor(0.015, dtype=torch.float64, requires_grad=True)
    loss = (A.residual(g, q, xy, a0) * w.to(DEV)).sum() + (A.forces(g, q, xy, a0) * c.to(DEV)).sum()
    loss.backward()
    flow.alpha0 = 0.015
    qr, xr, ar = O.residual_vjp(blocks, q0, flow, solver, w)
    qf, xf, af = O.forces_vjp(blocks, q0, flow, solver, c)
    _say("  q", _rel(q.grad.cpu(), qr + qf), "xy", _rel(xy.grad.cpu(), (xr[0] + xf[0]).reshape(-1)),
         "a0", float(a0.grad), float(ar + af))
    assert _rel(q.grad.cpu(), qr + qf) <= 1e-11
    assert _rel(xy.grad.cpu(), (xr[0] + xf[0]).reshape(-1)) <= 1e-11
    assert abs(float(a0.grad) - float(ar + af)) <= 1e-11 * abs(float(ar + af))
