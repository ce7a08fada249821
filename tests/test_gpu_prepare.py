"""hb_prepare: the scratch of the adjoints and of the time-domain march
allocated ahead, so that the calls themselves allocate nothing.  Checked by
the device's free memory (unchanged across a prepared call, reduced by an
unprepared first call) and by capturing prepared calls into a HIP graph,
whose replays (with eager work in between) must equal the eager results bit
for bit; the node-coordinate adjoints to rounding, as their ghost-side terms
are FP64 atomic adds whose order can differ from run to run."""
import sys

import pytest
import torch

from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _adjoint_case():
    p = synth.make_problem("naca256x128_hh64")
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    q = torch.as_tensor(synth.initial_state(p)).to(DEV)
    gen = torch.Generator(device="cpu").manual_seed(11)
    rbar = torch.randn(g.n_state, generator=gen, dtype=torch.float64).to(DEV)
    outs = (torch.empty_like(q), torch.empty(g.n_xy, dtype=torch.float64, device=DEV),
            torch.empty(1, dtype=torch.float64, device=DEV))
    return g, q, rbar, outs


def test_unprepared_adjoint_allocates_on_its_first_call():
    g, q, rbar, (qbar, xybar, fbar) = _adjoint_case()
    f0 = _free()
    g.residual_adjoint(q, rbar, qbar, xybar, fbar)
    f1 = _free()
    _say("  first unprepared call took", (f0 - f1) / 2 ** 20, "MiB")
    assert f1 < f0
    g.close()


def test_prepared_adjoint_allocates_nothing_and_captures():
    g, q, rbar, (qbar, xybar, fbar) = _adjoint_case()
    f0 = _free()
    g.prepare(hb.HB_PREPARE_ADJOINT)
    f1 = _free()
    assert f1 < f0                                  # the scratch is allocated here
    g.residual_adjoint(q, rbar, qbar, xybar, fbar)
    assert _free() == f1                            # and not by the call
    ref = (qbar.clone(), xybar.clone(), fbar.clone())
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        g.residual_adjoint(q, rbar, qbar, xybar, fbar)
    torch.cuda.synchronize()
    for k in range(3):
        for t in (qbar, xybar, fbar):
            t.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(qbar, ref[0]) and torch.equal(fbar, ref[2]), k
        d = float((xybar - ref[1]).norm() / ref[1].norm())
        _say("  replay", k, "xybar rel to the eager call", d)
        assert d <= 1e-14, (k, d)
        _ = (q * 2.0).sum().item()                  # eager work between replays
    g.close()


def test_prepared_adjoint_iteration_and_time_march_allocate_nothing():
    g, q, rbar, _ = _adjoint_case()
    g.prepare(hb.HB_PREPARE_ADJOINT_ITERATE)
    lam = torch.zeros_like(q)
    f0 = _free()
    g.adjoint_iterate(q, lam, rbar, 3)
    assert _free() == f0
    g.close()
    p = synth.make_problem("cyl_tiny")
    blk = p.blocks[0]
    b0 = synth.Block(blk.ni, blk.nj, 0, blk.xy, blk.bc)
    pt = synth.Problem("td", [b0], p.flow, synth.Solver(cfl=1.0, batched=1), 0, 21)
    gt = hb.Grid(pt.blocks, pt.flow, pt.solver, precision=0, batched=1)
    qt = torch.as_tensor(synth.initial_state(pt)).to(DEV)
    gt.prepare(hb.HB_PREPARE_TD)
    gt.td_march(qt.clone(), 0.0, 1e-3, 1)           # first launches of the residual path
    qa = qt.clone()
    f1 = _free()
    gt.td_march(qa, 0.0, 1e-3, 4)
    assert _free() == f1
    # captured: the same four steps on a copy, replayed from the same start
    qb = qt.clone()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        gt.td_march(qb, 0.0, 1e-3, 4)
    for k in range(3):
        qb.copy_(qt)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(qb, qa), k
    gt.close()


def test_prepare_refusals():
    p = synth.make_problem("cyl_tiny")
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=1, batched=1)
    with pytest.raises(hb.HBError) as e:
        g.prepare(hb.HB_PREPARE_ADJOINT_ITERATE)
    assert e.value.code == hb.HB_ERR_UNSUPPORTED
    with pytest.raises(hb.HBError) as e:
        g.prepare(8)
    assert e.value.code == hb.HB_ERR_ARG
    g.prepare(hb.HB_PREPARE_ADJOINT | hb.HB_PREPARE_TD)   # forces adjoint and march: any precision
    g.close()
