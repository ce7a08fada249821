"""Pin the oracle's block cuts (halo exchange between glued blocks, the
paper's multi-block decomposition, §MPI Optimisations): a block cut into
pieces must give the residual, forces and pseudo-time iteration of the uncut
block, whose periodic, wall, wake-cut and farfield ghosts are pinned
elsewhere.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import synth

CASES = [("cyl_tiny", 2, 2), ("cyl_tiny", 3, 1), ("naca_tiny", 1, 2), ("cyl_tiny", 1, 3)]


def _setup(name, pi, pj):
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.03
    sp, perm = synth.split_problem(p, pi, pj)
    blocks, flow, solver = O.from_synth(p)
    sblocks, _, _ = O.from_synth(sp)
    q = torch.as_tensor(synth.initial_state(p))
    return p, sp, torch.as_tensor(perm), blocks, sblocks, flow, solver, q


@pytest.mark.parametrize("name,pi,pj", CASES)
def test_split_residual_equals_uncut(name, pi, pj):
    p, sp, perm, blocks, sblocks, flow, solver, q = _setup(name, pi, pj)
    assert len(sp.blocks) == pi * pj and sp.n_state == p.n_state
    assert torch.equal(torch.sort(perm).values, torch.arange(p.n_state))
    r = O.residual_all(blocks, q, flow, solver)
    rs = O.residual_all(sblocks, q[perm], flow, solver, sp.cuts)
    assert float((rs - r[perm]).abs().max()) <= 1e-13 * float(r.abs().max())


@pytest.mark.parametrize("name,pi,pj", CASES[:3])
def test_split_forces_and_iteration_equal_uncut(name, pi, pj):
    p, sp, perm, blocks, sblocks, flow, solver, q = _setup(name, pi, pj)
    cf = torch.cat([c.reshape(-1) for c in O.forces(blocks, q, flow, solver)])
    cfs = torch.cat([c.reshape(-1) for c in O.forces(sblocks, q[perm], flow, solver,
                                                      cuts=sp.cuts)])
    assert float((cf - cfs).abs().max()) <= 1e-13 * float(cf.abs().max())
    q1, n1 = O.rk_iterate(blocks, q, flow, solver, 1)
    q2, n2 = O.rk_iterate(sblocks, q[perm], flow, solver, 1, sp.cuts)
    assert float((q2 - q1[perm]).abs().max()) <= 1e-14 * float(q1.abs().max())
    assert abs(float(n1[0]) - float(n2[0])) <= 1e-13 * float(n1[0])


def test_split_vjp_equals_uncut():
    p, sp, perm, blocks, sblocks, flow, solver, q = _setup("cyl_tiny", 2, 2)
    rbar = torch.randn(q.shape, generator=torch.Generator().manual_seed(4), dtype=O.DT)
    qb, xb, ab = O.residual_vjp(blocks, q, flow, solver, rbar)
    qbs, xbs, abs_ = O.residual_vjp(sblocks, q[perm], flow, solver, rbar[perm], sp.cuts)
    assert float((qbs - qb[perm]).abs().max()) <= 1e-12 * float(qb.abs().max())
    assert abs(float(ab) - float(abs_)) <= 1e-12 * abs(float(ab))
    # node bars: a node shared by several pieces collects from each of them
    ni, nj = p.blocks[0].ni, p.blocks[0].nj
    acc = torch.zeros_like(xb[0])
    ib = [round(k * ni / 2) for k in range(3)]
    jb = [round(k * nj / 2) for k in range(3)]
    for k, x in enumerate(xbs):
        pi, pj = k % 2, k // 2
        acc[:, jb[pj]:jb[pj + 1] + 1, ib[pi]:ib[pi + 1] + 1] += x
    # the periodic seam i = 0 / i = ni is one node twice in the uncut block
    assert float((acc - xb[0]).abs().max()) <= 1e-12 * float(xb[0].abs().max())


def test_cut_validation():
    p = synth.make_problem("cyl_tiny")
    sp, _ = synth.split_problem(p, 2, 1)
    sblocks, _, _ = O.from_synth(sp)
    with pytest.raises(ValueError):
        O.cut_partners(sblocks, [])                          # CUT side without a cut
    with pytest.raises(ValueError):
        O.cut_partners(sblocks, [(0, 1, 1, 2), (1, 1, 0, 0)])  # imax glued to a jmin
    with pytest.raises(ValueError):
        synth.split_problem(synth.make_problem("naca_tiny"), 2, 1)


# General cuts: segments of sides, any pairing of sides, reversed segments.
def _general(name, make):
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.03
    sp, perm = make(p)
    blocks, flow, solver = O.from_synth(p)
    sblocks, _, _ = O.from_synth(sp)
    q = torch.as_tensor(synth.initial_state(p))
    return p, sp, torch.as_tensor(perm), blocks, sblocks, flow, solver, q


GENERAL = [("naca_tiny", synth.split_c_grid),                     # reversed wake cut
           ("cyl_tiny", lambda p: synth.split_partial(p)),         # two segments per side
           ("cyl_tiny", lambda p: synth.rotate_block(synth.split_problem(p, 2, 1)[0], 1))]


@pytest.mark.parametrize("name,make", GENERAL, ids=["c_grid_3", "partial", "rotated"])
def test_general_cuts_residual_and_iteration_equal_uncut(name, make):
    """A C-grid cut into wake and profile blocks (the wake cut a reversed
    cut between two blocks), an O-grid whose right half is glued to two
    blocks per side, and an O-grid piece turned a quarter in index space
    (imax glued to a jmax): each gives the uncut block's residual and
    iteration, cell for cell."""
    p, sp, perm, blocks, sblocks, flow, solver, q = _general(name, make)
    if name == "cyl_tiny" and len(sp.blocks) == 2:
        # the rotated piece: perm maps the split layout, compose with the split's
        sp0, perm0 = synth.split_problem(p, 2, 1)
        perm = torch.as_tensor(perm0)[perm]
    assert torch.equal(torch.sort(perm).values, torch.arange(p.n_state))
    assert all(float(O.metrics(b.xy)[2].min()) > 0 for b in sblocks)
    r = O.residual_all(blocks, q, flow, solver)
    rs = O.residual_all(sblocks, q[perm], flow, solver, sp.cuts)
    assert float((rs - r[perm]).abs().max()) <= 1e-13 * float(r.abs().max())
    q1, n1 = O.rk_iterate(blocks, q, flow, solver, 1)
    q2, n2 = O.rk_iterate(sblocks, q[perm], flow, solver, 1, sp.cuts)
    assert float((q2 - q1[perm]).abs().max()) <= 1e-14 * float(q1.abs().max())
    assert abs(float(n1[0]) - float(n2[0])) <= 1e-13 * float(n1[0])


@pytest.mark.parametrize("name,make", GENERAL[:2], ids=["c_grid_3", "partial"])
def test_general_cuts_forces_equal_uncut(name, make):
    p, sp, perm, blocks, sblocks, flow, solver, q = _general(name, make)
    cf = torch.cat([c.reshape(-1) for c in O.forces(blocks, q, flow, solver)])
    cfs = torch.cat([c.reshape(-1) for c in O.forces(sblocks, q[perm], flow, solver, cuts=sp.cuts)])
    assert float((cf - cfs).abs().max()) <= 1e-13 * float(cf.abs().max())


def test_c_grid_in_three_blocks_vjp_equals_single():
    p, sp, perm, blocks, sblocks, flow, solver, q = _general("naca_tiny", synth.split_c_grid)
    rbar = torch.randn(q.shape, generator=torch.Generator().manual_seed(5), dtype=O.DT)
    qb, _, ab = O.residual_vjp(blocks, q, flow, solver, rbar)
    qbs, _, abs_ = O.residual_vjp(sblocks, q[perm], flow, solver, rbar[perm], sp.cuts)
    assert float((qbs - qb[perm]).abs().max()) <= 1e-12 * float(qb.abs().max())
    assert abs(float(ab) - float(abs_)) <= 1e-12 * abs(float(ab))


def test_general_cut_validation():
    p = synth.make_problem("cyl_tiny")
    sp, _ = synth.split_partial(p)
    sblocks, _, _ = O.from_synth(sp)
    O.cut_partners(sblocks, sp.cuts)
    with pytest.raises(ValueError):                            # a side half covered
        O.cut_partners(sblocks, sp.cuts[:-1])
    with pytest.raises(ValueError):                            # overlapping segments
        O.cut_partners(sblocks, sp.cuts + [(2, 1, 5, 1, 0, 0, 2, 0)])
    with pytest.raises(ValueError):                            # leaves the side
        O.cut_partners(sblocks, sp.cuts[:-1] + [(2, 1, 10, 1, 0, 0, 12, 0)])
    # a planted mistake: the wake cut not reversed changes the residual
    pc = synth.make_problem("naca_tiny")
    sc, perm = synth.split_c_grid(pc)
    cb, flow, solver = O.from_synth(sc)
    q = torch.as_tensor(synth.initial_state(pc))[torch.as_tensor(perm)]
    good = O.residual_all(cb, q, flow, solver, sc.cuts)
    bad_cuts = sc.cuts[:2] + [tuple(sc.cuts[2][:7]) + (0,)]
    bad = O.residual_all(cb, q, flow, solver, bad_cuts)
    assert float((good - bad).abs().max()) > 1e-6 * float(good.abs().max())
