"""The precision policy on a converged HB solution: flux, source and time
step in FP32 (perturbation form) with the state, update, norms and forces in
FP64 must reproduce the FP64 path's force harmonics within the stated 1e-4
(relative 2-norm over each coefficient's harmonic vector).  The FP64 end
state is checked against the oracle's residual, so "converged" is pinned
independently of the GPU path."""
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
