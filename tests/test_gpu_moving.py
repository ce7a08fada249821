"""GPU parity of the rigidly heaving and pitching grid (plain FP64 path,
hb_set_motion) against the moving-grid oracle on the same seeded inputs:
residual, pseudo-time iterations and loads, plus the entry points' refusal
of what a moving grid does not support."""
import sys

import pytest
import torch

from oracle import hb_moving as M
from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
# large enough that the motion terms are a sizeable part of every flux
MOT = dict(pitch_amp=0.3, pitch_phase=0.5, heave_amp=1.5, x_pivot=0.25, y_pivot=0.05)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(blocks, x, ref):
    xs, rs = O.split(blocks, x), O.split(blocks, ref)
    out = []
    for v in range(4):
        num = sum(float(((a[:, v] - b[:, v]) ** 2).sum()) for a, b in zip(xs, rs))
        den = sum(float((b[:, v] ** 2).sum()) for b in rs)
        out.append((num / den) ** 0.5)
    return max(out)


def _elem(blocks, x, ref):
    xs, rs = O.split(blocks, x), O.split(blocks, ref)
    worst = 0.0
    for v in range(4):
        scale = max(float(b[:, v].abs().max()) for b in rs)
        worst = max(worst, max(float((a[:, v] - b[:, v]).abs().max()) for a, b in zip(xs, rs)) / scale)
    return worst


def _setup(name):
    p = synth.make_problem(name)
    blocks, flow, solver = O.from_synth(p)
    q = torch.as_tensor(synth.initial_state(p))
    return p, blocks, flow, solver, q


@pytest.mark.parametrize("name", ["cyl_tiny", "naca_tiny", "batch_tiny"])
def test_moving_residual(name):
    _say("case", name, "moving-grid residual")
    p, blocks, flow, solver, q = _setup(name)
    ref = M.moving_residual_all(blocks, q, flow, solver, M.OMotion(**MOT))
    fixed = O.residual_all(blocks, q, flow, solver)
    assert _rel(blocks, fixed, ref) > 1e-2          # the motion matters
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    g.set_motion(**MOT)
    r = g.residual(q.to(DEV)).cpu()
    torch.cuda.synchronize()
    assert _rel(blocks, r, ref) <= 1e-12
    assert _elem(blocks, r, ref) <= 1e-11


@pytest.mark.parametrize("name", ["cyl_tiny", "batch_tiny"])
def test_moving_rk_iterate(name):
    _say("case", name, "moving-grid RK")
    p, blocks, flow, solver, q = _setup(name)
    n_it = 3
    qref, nref = M.moving_rk_iterate(blocks, q, flow, solver, M.OMotion(**MOT), n_it)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    g.set_motion(**MOT)
    qd = q.to(DEV)
    norms = torch.zeros(n_it, dtype=torch.float64, device=DEV)
    g.rk_iterate(qd, n_it, norms)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    assert _rel(blocks, qd.cpu() - q, qref - q) <= 1e-11
    assert torch.allclose(norms.cpu(), nref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("name", ["cyl_tiny", "naca_tiny", "batch_tiny"])
def test_moving_forces(name):
    _say("case", name, "moving-grid loads")
    p, blocks, flow, solver, q = _setup(name)
    ref = torch.cat([c.reshape(-1) for c in M.moving_forces(blocks, q, flow, solver, M.OMotion(**MOT))])
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    g.set_motion(**MOT)
    cf = g.forces(q.to(DEV)).cpu()
    torch.cuda.synchronize()
    fixed = torch.cat([c.reshape(-1) for c in O.forces(blocks, q, flow, solver)])
    assert float((fixed - ref).abs().max()) > 1e-3 * float(ref.abs().max())
    assert float((cf - ref).abs().max()) <= 1e-11 * float(ref.abs().max())


def test_moving_full_size_sampled_block():
    """The bench's moving-grid configuration (all 32 blocks of the batch, one
    plain-path call): blocks without cuts are independent, so the smallest
    block's residual is checked against the oracle element by element."""
    p = synth.make_problem("batch32_mixed")
    _say("case batch32_mixed moving-grid residual, sampled block")
    q = torch.as_tensor(synth.initial_state(p))
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    g.set_motion(**MOT)
    r = g.residual(q.to(DEV)).cpu()
    torch.cuda.synchronize()
    blocks, flow, solver = O.from_synth(p)
    k = min(range(len(blocks)), key=lambda i: blocks[i].ns * blocks[i].ni * blocks[i].nj)
    off = sum(b.ns * 4 * b.ni * b.nj for b in blocks[:k])
    b = blocks[k]
    n = b.ns * 4 * b.ni * b.nj
    qb = q[off:off + n].reshape(b.ns, 4, b.nj, b.ni)
    ref = M.moving_residual(b, qb, flow, solver, M.OMotion(**MOT)).reshape(-1)
    assert _rel([b], r[off:off + n], ref) <= 1e-12
    assert bool(torch.isfinite(r).all())


def test_clearing_motion_restores_fixed_grid_bitwise():
    p, blocks, flow, solver, q = _setup("cyl_tiny")
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    qd = q.to(DEV)
    r0 = g.residual(qd).clone()
    g.set_motion(**MOT)
    r1 = g.residual(qd).clone()
    g.set_motion()
    r2 = g.residual(qd).clone()
    torch.cuda.synchronize()
    assert not torch.equal(r0, r1)
    assert torch.equal(r0, r2)


def test_moving_grid_refusals():
    p, blocks, flow, solver, q = _setup("cyl_tiny")
    gb = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    with pytest.raises(hb.HBError) as e:
        gb.set_motion(**MOT)
    assert e.value.code == hb.HB_ERR_UNSUPPORTED
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=0)
    with pytest.raises(hb.HBError) as e:
        g.set_motion(pitch_amp=float("nan"))
    assert e.value.code == hb.HB_ERR_ARG
    g.set_motion(**MOT)
    qd = q.to(DEV)
    with pytest.raises(hb.HBError) as e:
        g.residual_adjoint(qd, torch.ones_like(qd))
    assert e.value.code == hb.HB_ERR_UNSUPPORTED
    with pytest.raises(hb.HBError) as e:
        g.forces_adjoint(qd, torch.ones(g.n_forces, dtype=torch.float64, device=DEV))
    assert e.value.code == hb.HB_ERR_UNSUPPORTED
