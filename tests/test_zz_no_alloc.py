"""hb_td_march_noalloc (the time-domain march for callers that cannot
allocate: its scratch lives in a static per-device array) against
hb_td_march on the same grids and inputs, on two calls in a row, the second
with a smaller grid, plus the refusal of a state larger than the static
scratch."""
import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _o_problem(ni, nj):
    blk = synth.Block(ni, nj, 0, synth.o_grid(ni, nj, r_out=6.0),
                      (synth.PERIODIC, synth.PERIODIC, synth.WALL, synth.FARFIELD))
    flow = synth.Flow(mach=0.3, reynolds=20.0, alpha_amp=0.03, k_red=1.0)
    return synth.Problem("noalloc_o", [blk], flow, synth.Solver(cfl=1.0), 0, 31)


def _c_problem(ni, nj):
    blk = synth.c_block(ni, nj, 0)
    flow = synth.flow_airfoil()
    flow.alpha_amp = 0.02
    return synth.Problem("noalloc_c", [blk], flow, synth.Solver(cfl=1.0), 0, 32)


def _both(p, batched, n_steps):
    blocks, flow, _ = O.from_synth(p)
    q0 = torch.as_tensor(synth.initial_state(p))
    b = blocks[0]
    dt = 0.5 * float(O.local_dt(b, q0.reshape(1, 4, b.nj, b.ni), flow,
                                O.OSolver(cfl=1.0)).min())
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=batched)
    qa = q0.to(DEV)
    qb = q0.to(DEV)
    g.td_march(qa, 0.3, dt, n_steps)
    g.td_march_noalloc(qb, 0.3, dt, n_steps)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    assert float((qa - q0.to(DEV)).abs().max()) > 0
    g.close()
    return qa.cpu(), qb.cpu()


def test_noalloc_march_matches_allocating_march():
    # first call: batched FP64 O-grid 64x32; second: smaller plain FP64 C-grid
    for p, batched, n in ((_o_problem(64, 32), 1, 20), (_c_problem(40, 12), 0, 15)):
        _say("case", p.name, p.blocks[0].ni, "x", p.blocks[0].nj, "batched", batched)
        qa, qb = _both(p, batched, n)
        _say("  max |noalloc - alloc| =", float((qa - qb).abs().max()))
        assert torch.equal(qa, qb)


def test_noalloc_march_refuses_large_state():
    # 4 x 1024 x 520 doubles > 2^21: beyond the static scratch
    p = _c_problem(1024, 520)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    q = torch.zeros(g.n_state, dtype=torch.float64, device=DEV)
    with pytest.raises(hb.HBError) as e:
        g.td_march_noalloc(q, 0.0, 1e-3, 1)
    assert e.value.code == hb.HB_ERR_ARG
    assert "static scratch" in str(e.value)
    g.close()
