"""The time-domain march on the GPU (hb_td_march): parity with the oracle's
fourth-order physical-time march, and the HB-vs-time-domain check on the
GPU at a larger grid than the oracle's own pin: converged N_H = 1, 2, 3
snapshots against a periodic time-domain march sampled at the same phases
(the difference is the response's content above harmonic N_H)."""
import math

import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _problem(kind, n_harm, alpha_amp, ni, nj):
    if kind == "o":
        blk = synth.Block(ni, nj, n_harm, synth.o_grid(ni, nj, r_out=6.0),
                          (synth.PERIODIC, synth.PERIODIC, synth.WALL, synth.FARFIELD))
        flow = synth.Flow(mach=0.3, reynolds=20.0, alpha_amp=alpha_amp, k_red=1.0)
    else:
        blk = synth.c_block(ni, nj, n_harm)
        flow = synth.flow_airfoil()
        flow.alpha_amp = alpha_amp
    return synth.Problem("td_%s" % kind, [blk], flow, synth.Solver(cfl=1.0), 0, 21)


@pytest.mark.parametrize("kind", ["o", "c"])
@pytest.mark.parametrize("prec,batched", [(0, 0), (0, 1), (1, 1)])
def test_td_march_matches_oracle(kind, prec, batched):
    _say("td march", kind, prec, batched)
    p = _problem(kind, 0, 0.03, 24 if kind == "o" else 72, 12 if kind == "o" else 20)
    blocks, flow, solver = O.from_synth(p)
    q0 = torch.as_tensor(synth.initial_state(p))
    b = blocks[0]
    qb = q0.reshape(1, 4, b.nj, b.ni)
    dt = 0.5 * float(O.local_dt(b, qb, flow, O.OSolver(cfl=1.0)).min())
    t0, n = 0.7, 12
    ref = O.td_march(b, qb, flow, solver, dt, n, t0).reshape(-1)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=prec, batched=batched)
    q = q0.to(DEV)
    g.td_march(q, t0, dt, n)
    torch.cuda.synchronize()
    d = (q.cpu() - q0)
    rel = float((d - (ref - q0)).norm() / (ref - q0).norm())
    _say("  rel error of the change", rel)
    assert rel <= (1e-11 if prec == 0 else 1e-5)
    # the grid's own far field is restored: its residual is unchanged
    r1 = g.residual(q0.to(DEV)).cpu()
    rref = O.residual_all(blocks, q0, flow, solver)
    assert float((r1 - rref).norm() / rref.norm()) <= (1e-12 if prec == 0 else 1e-5)


def test_td_rejects_hb_grids():
    p = synth.make_problem("cyl_tiny")
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    q = torch.as_tensor(synth.initial_state(p)).to(DEV)
    with pytest.raises(hb.HBError):
        g.td_march(q, 0.0, 1e-3, 1)


def _converge_hb(p, q, n_iter):
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    norms = torch.zeros(n_iter, dtype=torch.float64, device=DEV)
    g.rk_iterate(q, n_iter, norms)
    torch.cuda.synchronize()
    assert g.status() == hb.HB_OK
    n = norms.cpu()
    return float(n[-1] / n[0])


def _td_periodic_gpu(p0, q0, T, steps, samples, tol, max_periods=80):
    """hb_td_march period by period from q0 until the state at phase 0 changes
    by less than tol over a period; the last period sampled at phases
    k/samples, [samples][4][nj][ni] on the host."""
    g = hb.Grid(p0.blocks, p0.flow, p0.solver, precision=0, batched=1)
    dt, per = T / steps, steps // samples
    qt, t = q0.clone(), 0.0
    for k in range(max_periods):
        start, snaps = qt.clone(), []
        for _ in range(samples):
            snaps.append(qt.clone())
            g.td_march(qt, t, dt, per)
            t += dt * per
        change = float((qt - start).abs().max())
        if change < tol:
            _say("  time-domain march periodic after", k + 1, "periods")
            return torch.stack(snaps).cpu()
    raise AssertionError("time-domain march not periodic: change %g" % change)


@pytest.mark.parametrize("ni,nj,n_harms", [(16, 8, (1, 2, 3)), (48, 24, (1,))])
def test_hb_matches_time_domain_march_on_gpu(ni, nj, n_harms):
    """Check (e) on the GPU: the converged HB snapshots against the
    time-domain march, marched until periodic (change below 1e-12 per
    period) and sampled at the same phases.  The difference is the
    response's content above harmonic N_H: a small fraction of the unsteady
    response at N_H = 1, shrinking about four-fold when A halves.  On the
    16x8 grid of the oracle's own pin it falls by more than an order of
    magnitude per added harmonic and like A^(N_H+1) (ratios 8 and 16 for
    N_H = 2 and 3).  On the 48x24 grid only N_H = 1 is checked: there the
    Roe eigenvalue modulus |q_n| of the faces on the stagnation line
    (theta = 0 and pi) changes sign twice per period, a kink of the discrete
    operator whose harmonics fall off slowly and scale like A^2, which puts
    a floor of about 5e-6 under the N_H = 2 difference at A = 1e-3."""
    # steady mean flow first (N_H = 0, no forcing), then the HB solutions
    ps = _problem("o", 0, 0.0, ni, nj)
    ps.solver.graph_iters = 50
    qs = torch.as_tensor(synth.initial_state(ps)).to(DEV)
    drop = _converge_hb(ps, qs, 20000)
    _say("  steady drop", drop)
    blocks, flow, _ = O.from_synth(ps)
    T = 2 * math.pi / flow.omega
    dtmin = 0.5 * float(O.local_dt(blocks[0], qs.cpu().reshape(1, 4, nj, ni), flow,
                                   O.OSolver(cfl=1.0)).min())
    steps = 105 * int(math.ceil(T / dtmin / 105))
    err, amp = {}, {}
    for A in (1e-3, 5e-4):
        td = _td_periodic_gpu(_problem("o", 0, A, ni, nj), qs, T, steps, 105, 1e-12)
        for nh in n_harms:
            ns = 2 * nh + 1
            p1 = _problem("o", nh, A, ni, nj)
            p1.solver.graph_iters = 50
            q = qs.reshape(1, -1).repeat(ns, 1).reshape(-1).contiguous()
            drop = _converge_hb(p1, q, 40000)
            assert drop <= 1e-9, drop
            qh = q.cpu().reshape(ns, 4, nj, ni)
            ref = td[[n * 105 // ns for n in range(ns)]].reshape(ns, 4, nj, ni)
            err[(A, nh)] = (ref - qh).abs().max().item()
            amp[(A, nh)] = (qh - qh.mean(0, keepdim=True)).abs().max().item()
            _say("  A", A, "N_H", nh, "HB drop", drop, "err", err[(A, nh)],
                 "amp", amp[(A, nh)])
    for A in (1e-3, 5e-4):
        assert err[(A, 1)] < 0.05 * amp[(A, 1)], (err, amp)
    assert 3.0 < err[(1e-3, 1)] / err[(5e-4, 1)] < 5.0, err
    if 2 in n_harms:
        for A in (1e-3, 5e-4):
            assert err[(A, 2)] < err[(A, 1)] / 10, err
            assert err[(A, 3)] < err[(A, 2)] / 5, err
        assert 6.0 < err[(1e-3, 2)] / err[(5e-4, 2)] < 10.0, err
        assert 11.0 < err[(1e-3, 3)] / err[(5e-4, 3)] < 22.0, err
