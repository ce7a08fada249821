"""Batched grids of any state size: the fused kernel's halo loads take
64-bit element offsets when the FP64 state reaches 4 GiB (and with
batched = 2 at any size).  On small grids the 64-bit variant must give the
32-bit variant's results bit for bit (only the addressing differs) and the
oracle's; above 4 GiB, blocks whose halo lies beyond the 32-bit range (a
glued pair at the two ends of the state, separated by filler blocks) must
match the oracle's residual and iteration of the pair."""
import sys

import numpy as np
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


def _rel(blocks, x, ref):
    xs, rs = O.split(blocks, x), O.split(blocks, ref)
    out = []
    for v in range(4):
        num = sum(float(((a[:, v] - b[:, v]) ** 2).sum()) for a, b in zip(xs, rs))
        den = sum(float((b[:, v] ** 2).sum()) for b in rs)
        out.append((num / den) ** 0.5)
    return max(out)


def _split(name, pi, pj):
    p = synth.make_problem(name)
    if pi * pj == 1:
        return p, torch.as_tensor(synth.initial_state(p))
    sp, perm = synth.split_problem(p, pi, pj)
    q = torch.as_tensor(synth.initial_state(p))[torch.as_tensor(perm)].contiguous()
    return sp, q


def _run(p, q, prec, batched, motion=None, n_it=2):
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=prec, batched=batched)
    if motion:
        g.set_motion(**motion)
    r = g.residual(q.to(DEV)).cpu()
    qd = q.to(DEV)
    norms = torch.zeros(n_it, dtype=torch.float64, device=DEV)
    g.rk_iterate(qd, n_it, norms)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    g.close()
    return r, qd.cpu(), norms.cpu()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,pi,pj", [("batch_tiny", 1, 1), ("cyl_tiny", 2, 2), ("naca_tiny", 1, 2)])
def test_64bit_addressing_matches_32bit_and_oracle(name, pi, pj, prec):
    _say("case", name, pi, pj, "precision", prec)
    p, q = _split(name, pi, pj)
    blocks, flow, solver = O.from_synth(p)
    r32, q32, n32 = _run(p, q, prec, 1)
    r64, q64, n64 = _run(p, q, prec, 2)
    assert torch.equal(r32, r64) and torch.equal(q32, q64) and torch.equal(n32, n64)
    ref = O.residual_all(blocks, q, flow, solver, p.cuts)
    qref, _ = O.rk_iterate(blocks, q, flow, solver, 2, p.cuts)
    err, qerr = _rel(blocks, r64, ref), _rel(blocks, q64 - q, qref - q)
    _say("  residual", err, "state change", qerr)
    assert err <= (1e-12 if prec == 0 else 1e-5)
    assert qerr <= (1e-11 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_64bit_addressing_moving_grid(prec):
    p, q = _split("cyl_tiny", 2, 2)
    blocks, flow, solver = O.from_synth(p)
    r32, q32, _ = _run(p, q, prec, 1, MOT)
    r64, q64, _ = _run(p, q, prec, 2, MOT)
    assert torch.equal(r32, r64) and torch.equal(q32, q64)
    ref = M.moving_residual_all(blocks, q, flow, solver, M.OMotion(**MOT), p.cuts)
    err = _rel(blocks, r64, ref)
    _say("  moving residual", err)
    assert err <= (1e-12 if prec == 0 else 1e-5)


def _free_stream(flow, n_harm):
    """Free-stream conserved variables [ns][4] of each snapshot."""
    tiny = synth.Problem("fs", [synth.Block(4, 4, n_harm, synth.o_grid(4, 4),
                                            (synth.PERIODIC, synth.PERIODIC, synth.WALL,
                                             synth.FARFIELD))], flow, synth.Solver(), 0, 1)
    q = synth.initial_state(tiny, amplitude=0.0).reshape(2 * n_harm + 1, 4, 4, 4)
    return torch.as_tensor(q[:, :, 0, 0].copy())


@pytest.mark.parametrize("prec", [1, 0])
def test_state_above_4_gib(prec):
    """A cylinder split into two glued halves A and B, placed first and last
    in a batch whose FP64 state is 4.5 GiB (eight 2048x1024 N_H = 4 filler
    blocks in between): A's halo across the cut lies beyond 4 GiB of it, B's
    whole state beyond 4 GiB of the array's start.  Residual and one
    iteration of A and B against the oracle's for the glued pair."""
    pair, qpair = _split("cyl_tiny", 2, 1)
    assert len(pair.blocks) == 2
    A, B = pair.blocks
    ni, nj, nh = 2048, 1024, 4
    xy = synth.o_grid(ni, nj)
    nf = 8
    fillers = [synth.Block(ni, nj, nh, xy, (synth.PERIODIC, synth.PERIODIC, synth.WALL, synth.FARFIELD),
                           0, 1 + k) for k in range(nf)]        # a body of its own each
    filler = fillers[0]
    blocks = [A] + fillers + [B]
    last = nf + 1
    cuts = [(last if a == 1 else a, sa, last if b == 1 else b, sb) for a, sa, b, sb in pair.cuts]
    p = synth.Problem("large", blocks, pair.flow, pair.solver, 0, 21, cuts=cuts)
    n_a = A.ns * 4 * A.ni * A.nj
    n_b = B.ns * 4 * B.ni * B.nj
    n_f = filler.ns * 4 * ni * nj
    total = n_a + nf * n_f + n_b
    assert total * 8 > 4 * 2 ** 30 + 2 ** 28
    _say("state", total * 8 / 2 ** 30, "GiB, precision", prec)
    q = torch.empty(total, dtype=torch.float64, device=DEV)
    q[:n_a] = qpair[:n_a].to(DEV)
    q[total - n_b:] = qpair[n_a:].to(DEV)
    fs = _free_stream(pair.flow, nh).to(DEV)                       # [ns][4]
    for k in range(nf):
        o = n_a + k * n_f
        q[o:o + n_f].view(filler.ns, 4, ni * nj).copy_(fs[:, :, None].expand(filler.ns, 4, ni * nj))
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=prec, batched=1)
    r = g.residual(q)
    ra = torch.cat([r[:n_a], r[total - n_b:]]).cpu()
    fr = float(r[n_a:total - n_b].abs().max())
    del r
    q1 = q.clone()
    g.rk_iterate(q1, 1)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    qa = torch.cat([q1[:n_a], q1[total - n_b:]]).cpu()
    del q1
    g.close()
    pb, flow, solver = O.from_synth(pair)
    ref = O.residual_all(pb, qpair, flow, solver, pair.cuts)
    qref, _ = O.rk_iterate(pb, qpair, flow, solver, 1, pair.cuts)
    err, qerr = _rel(pb, ra, ref), _rel(pb, qa - qpair, qref - qpair)
    _say("  residual of the glued pair", err, "state change", qerr, "filler residual max", fr)
    assert err <= (1e-12 if prec == 0 else 1e-5)
    assert qerr <= (1e-11 if prec == 0 else 1e-5)
    assert np.isfinite(fr)
