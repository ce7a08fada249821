"""Parity at the configurations' own sizes and iteration counts: the
64x32 N_H = 1 cylinder after its 100 iterations and the four-block N_H = 2
airfoil (256x64, 128x64, 64x64 and 192x96 glued blocks of one C-grid)
after its 500, on the per-block plain FP64 path and the batched FP64 path,
against the FP64 oracle run through the same iterations.

- State after N iterations: the change from the initial state per
  variable within 1e-10 (relative 2-norm over all blocks, cells and
  snapshots); the residual norm of every iteration within 1e-10.
- Residual on the oracle's states after 1, 10 and N iterations: per
  variable within 1e-12, or four times the FP64 rounding floor of the
  residual on that state where that is larger (parity_util.fp64_floor).

The oracle trajectory is computed once per configuration: the glued blocks
together, the blocks of a grid without cuts one worker process each."""
import multiprocessing as mp
import os
import time

import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth
from parity_util import block_trajectory, fp64_floor, fp64_tolerance, per_var_errors

pytestmark = pytest.mark.gpu
DEV = "cuda"
_TRAJ = {}


def _say(*a):
    print(*a, flush=True)


def _trajectory(name):
    """Oracle states after 0, 1, 10 and N iterations and all N norms.
    Blocks glued by cuts iterate together; the blocks of a grid without
    cuts run on their own in worker processes, and the norm of an iteration
    is put together from the blocks' sums of squares."""
    if name in _TRAJ:
        return _TRAJ[name]
    p = synth.make_problem(name)
    blocks, flow, solver = O.from_synth(p)
    q = torch.as_tensor(synth.initial_state(p))
    marks = (1, 10, p.n_iter)
    nb = len(blocks)
    t0 = time.time()
    states = {0: q}
    if p.cuts:
        torch.set_num_threads(min(16, os.cpu_count() or 1))
        qq, done, parts = q, 0, []
        for m in marks:
            qq, nr = O.rk_iterate(blocks, qq, flow, solver, m - done, p.cuts)
            states[m] = qq
            parts.append(nr)
            done = m
            _say("  oracle %s: %d iterations (%.0f s)" % (name, m, time.time() - t0))
        norms = torch.cat(parts)
    else:
        threads = max(1, (os.cpu_count() or 1) // nb)
        ctx = mp.get_context("spawn")
        with ctx.Pool(nb) as pool:
            res = pool.map(block_trajectory, [(name, k, marks, threads) for k in range(nb)])
        total = sum(b.ns * b.ni * b.nj for b in blocks)
        for m in marks:
            states[m] = O.join([r[0][m] for r in res])
        norms = torch.sqrt(sum(r[1] for r in res) / total)
    _say("  oracle %s: %d iterations of %d blocks (%.0f s)" % (name, p.n_iter, nb, time.time() - t0))
    _TRAJ[name] = (p, blocks, flow, solver, states, norms)
    return _TRAJ[name]


@pytest.mark.parametrize("name", ["cyl64x32_nh1", "naca4blk_nh2"])
@pytest.mark.parametrize("batched", [0, 1])
def test_state_after_full_iteration_count(name, batched):
    p, blocks, flow, solver, states, nref = _trajectory(name)
    n = p.n_iter
    _say("case", name, "batched", batched, n, "iterations")
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=0, batched=batched)
    q0 = states[0]
    qd = q0.to(DEV)
    norms = torch.zeros(n, dtype=torch.float64, device=DEV)
    g.rk_iterate(qd, n, norms)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    e = per_var_errors(blocks, qd.cpu() - q0, states[n] - q0)
    en = float(((norms.cpu() - nref).abs() / nref).max())
    _say("  state change rel per variable", e, "norms rel (max)", en,
         "norm drop", float(nref[-1] / nref[0]))
    assert max(e) <= 1e-10 and en <= 1e-10


@pytest.mark.parametrize("name", ["cyl64x32_nh1", "naca4blk_nh2"])
@pytest.mark.parametrize("batched", [0, 1])
def test_residual_on_oracle_states(name, batched):
    p, blocks, flow, solver, states, _ = _trajectory(name)
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=0, batched=batched)
    for it in (1, 10, p.n_iter):
        q = states[it]
        floor, ref = fp64_floor(blocks, q, flow, solver, p.cuts)
        tol = fp64_tolerance(floor)
        r = g.residual(q.to(DEV)).cpu()
        torch.cuda.synchronize()
        e = per_var_errors(blocks, r, ref)
        _say("  %s batched %d after %d: rel %s floor %s" % (name, batched, it,
             ["%.2e" % x for x in e], ["%.2e" % x for x in floor]))
        assert all(a <= t for a, t in zip(e, tol))


_MOVING = {}


def _moving_trajectory():
    """The four-block airfoil pitching 1 degree about its quarter chord on
    the moving grid (its 'pitching' taken literally: no incidence
    oscillation): the moving-grid oracle's state and norms after 10
    iterations."""
    if not _MOVING:
        import math
        from oracle import hb_moving as M
        torch.set_num_threads(min(16, os.cpu_count() or 1))
        p = synth.make_problem("naca4blk_nh2")
        p.flow.alpha_amp = 0.0
        blocks, flow, solver = O.from_synth(p)
        motion = dict(pitch_amp=math.radians(1.0), x_pivot=0.25)
        q = torch.as_tensor(synth.initial_state(p))
        t0 = time.time()
        q10, n10 = M.moving_rk_iterate(blocks, q, flow, solver, M.OMotion(**motion), 10, p.cuts)
        _say("  moving oracle: 10 iterations (%.0f s)" % (time.time() - t0))
        _MOVING.update(p=p, blocks=blocks, motion=motion, q=q, q10=q10, n10=n10)
    return _MOVING


@pytest.mark.parametrize("prec,batched", [(0, 0), (0, 1), (1, 1)])
def test_four_block_airfoil_pitching_on_a_moving_grid(prec, batched):
    """The four glued blocks at their size on the pitching grid: state and
    norms after 10 iterations against the moving-grid oracle (FP64 within
    1e-10, FP32 bulk within 1e-5), on the plain and the batched paths."""
    t = _moving_trajectory()
    p, blocks = t["p"], t["blocks"]
    _say("four-block airfoil pitching, prec", prec, "batched", batched)
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=prec, batched=batched)
    g.set_motion(**t["motion"])
    qd = t["q"].to(DEV)
    norms = torch.zeros(10, dtype=torch.float64, device=DEV)
    g.rk_iterate(qd, 10, norms)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    e = per_var_errors(blocks, qd.cpu() - t["q"], t["q10"] - t["q"])
    en = float(((norms.cpu() - t["n10"]).abs() / t["n10"]).max())
    _say("  state change rel per variable", e, "norms rel (max)", en)
    tol = 1e-10 if prec == 0 else 1e-5
    assert max(e) <= tol and en <= tol
    g.close()
