"""The precision policy on a converged HB solution: flux, source and time
step in FP32 (perturbation form) with the state, update, norms and forces in
FP64 must reproduce the FP64 path's force harmonics within the stated 1e-4
(relative 2-norm over each coefficient's harmonic vector).  The FP64 end
state is checked against the oracle's residual, so "converged" is pinned
independently of the GPU path.  At the 1024x512 N_H = 4 size the FP32 run
goes to its rounding floor and the FP64 run on from there to a 1e-8 drop."""
import os

import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _harmonics(cf, ns):
    """[body][n][3] -> per coefficient (cl, cd, cm) its real DFT vector."""
    c = cf.reshape(-1, ns, 3)[0]
    return [O.harmonics(c[:, k]) for k in range(3)]


@pytest.mark.parametrize("name,n_iter", [("naca_tiny_hh8", 12000)])
def test_converged_force_harmonics_fp32_vs_fp64(name, n_iter):
    p = synth.make_problem(name)
    p.solver.graph_iters = 50
    q0 = torch.as_tensor(synth.initial_state(p)).to(DEV)
    out = {}
    for prec in (0, 1):
        g = hb.Grid(p.blocks, p.flow, p.solver, precision=prec, batched=1)
        q = q0.clone()
        norms = torch.zeros(n_iter, dtype=torch.float64, device=DEV)
        g.rk_iterate(q, n_iter, norms)
        cf = g.forces(q)
        torch.cuda.synchronize()
        assert g.status() == hb.HB_OK
        n = norms.cpu()
        out[prec] = (q.cpu(), cf.cpu(), float(n[-1] / n[0]))
        g.close()
    _say("  drops: FP64", out[0][2], "FP32", out[1][2])
    assert out[0][2] <= 1e-11
    # the FP64 end state is a solution of the oracle's discrete equations
    blocks, flow, solver = O.from_synth(p)
    r = O.residual_all(blocks, out[0][0], flow, solver)
    r0 = O.residual_all(blocks, q0.cpu(), flow, solver)
    _say("  oracle |R*(q64)| / |R*(q0)| =", float(r.norm() / r0.norm()))
    assert float(r.norm() / r0.norm()) <= 1e-9
    ns = p.blocks[0].ns
    h64, h32 = _harmonics(out[0][1], ns), _harmonics(out[1][1], ns)
    for k, name_k in enumerate(("cl", "cd", "cm")):
        rel = float((h32[k] - h64[k]).norm() / h64[k].norm())
        _say("  %s harmonics FP64 %s  rel err FP32 %.3e" % (name_k, h64[k].tolist(), rel))
        assert rel <= 1e-4


def _iterate_until(g, q, chunk, max_iter, stop, label):
    """Iterate in chunks of `chunk`, calling stop(norms so far) after each;
    returns all norms."""
    hist = []
    norms = torch.zeros(chunk, dtype=torch.float64, device=DEV)
    done = 0
    while done < max_iter:
        g.rk_iterate(q, chunk, norms)
        torch.cuda.synchronize()
        assert g.status() == hb.HB_OK
        hist.append(norms.cpu().clone())
        done += chunk
        h = torch.cat(hist)
        _say("  %s: %d iterations, norm %.3e" % (label, done, float(h[-1])))
        if stop(h):
            break
    return torch.cat(hist)


def test_converged_force_harmonics_at_1024x512():
    """The precision configuration at its own size (1024x512 C-grid, N_H = 4):
    FP32 bulk from the seeded state until its residual drop reaches 1e-8 or
    stops falling (its window minimum over the last 20,000 iterations is
    not half the one before: the FP32 rounding floor), then the FP64 path
    from that state until the drop reaches 1e-8 (drops relative to the first
    FP64 norm from the seeded state).  The converged force harmonics of the
    two must agree within 1e-4, and the FP64 state must solve the oracle's
    discrete equations."""
    p = synth.make_problem("naca1024x512_nh4")
    p.solver.graph_iters = 50
    q0 = torch.as_tensor(synth.initial_state(p)).to(DEV)
    chunk = 5000
    g64 = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    n1 = torch.zeros(1, dtype=torch.float64, device=DEV)
    g64.rk_iterate(q0.clone(), 1, n1)
    ref = float(n1.cpu()[0])
    g32 = hb.Grid(p.blocks, p.flow, p.solver, precision=1, batched=1)
    q = q0.clone()

    def fp32_stop(h):
        if float(h[-1]) <= 1e-8 * ref:
            return True
        w = chunk * 4
        if len(h) < 2 * w:
            return False
        return float(h[-w:].min()) > 0.5 * float(h[-2 * w:-w].min())

    h32 = _iterate_until(g32, q, chunk, 160000, fp32_stop, "FP32")
    cf32 = g32.forces(q).cpu()
    drop32 = float(h32[-chunk:].min()) / ref
    h64 = _iterate_until(g64, q, chunk, 160000, lambda h: float(h[-1]) <= 1e-8 * ref, "FP64")
    cf64 = g64.forces(q).cpu()
    torch.cuda.synchronize()
    drop64 = float(h64[-1]) / ref
    _say("  drop reached: FP32 %.3e after %d iterations, FP64 %.3e after %d more"
         % (drop32, len(h32), drop64, len(h64)))
    assert drop64 <= 1e-8
    # the FP64 state solves the oracle's discrete equations: its oracle
    # residual is the drop reached, relative to the seeded state's
    torch.set_num_threads(min(16, os.cpu_count() or 1))
    blocks, flow, solver = O.from_synth(p)
    r = O.residual_all(blocks, q.cpu(), flow, solver)
    r0 = O.residual_all(blocks, q0.cpu(), flow, solver)
    ratio = float(r.norm() / r0.norm())
    _say("  oracle |R*(q64)| / |R*(q0)| =", ratio)
    assert ratio <= 1e-7
    ns = p.blocks[0].ns
    ha, hb_ = _harmonics(cf64, ns), _harmonics(cf32, ns)
    for k, name_k in enumerate(("cl", "cd", "cm")):
        rel = float((hb_[k] - ha[k]).norm() / ha[k].norm())
        _say("  %s harmonics FP64 %s  rel err FP32 %.3e" % (name_k, ha[k].tolist(), rel))
        assert rel <= 1e-4
