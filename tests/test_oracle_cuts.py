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


# partly glued sides: a C-grid cut where wake and profile share a piece's
# jmin (CUT_WALL sides with one or two wake segments), in two layers
PIECES = lambda p: synth.split_c_grid_at(p, [10, 40, 60], [8])


def test_partly_glued_c_grid_equals_single_block():
    """naca_tiny (72 x 20, wake 18) cut at i = 10, 40, 60 and j = 8: the
    bottom pieces' jmin sides are wake only (CUT), wake and profile
    (CUT_WALL, one with two wake segments to two pieces) and profile only
    (WALL).  Residual, loads, one iteration and the reverse products equal
    the single block's."""
    p, sp, perm, blocks, sblocks, flow, solver, q = _general("naca_tiny", PIECES)
    kinds = [b.bc[2] for b in sp.blocks[:4]]
    assert kinds == [synth.CUT, synth.CUT_WALL, synth.CUT_WALL, synth.CUT]
    assert torch.equal(torch.sort(perm).values, torch.arange(p.n_state))
    r = O.residual_all(blocks, q, flow, solver)
    rs = O.residual_all(sblocks, q[perm], flow, solver, sp.cuts)
    assert float((rs - r[perm]).abs().max()) <= 1e-13 * float(r.abs().max())
    cf = torch.cat([c.reshape(-1) for c in O.forces(blocks, q, flow, solver)])
    cfs = torch.cat([c.reshape(-1) for c in O.forces(sblocks, q[perm], flow, solver, cuts=sp.cuts)])
    assert float((cf - cfs).abs().max()) <= 1e-13 * float(cf.abs().max())
    q1, n1 = O.rk_iterate(blocks, q, flow, solver, 1)
    q2, n2 = O.rk_iterate(sblocks, q[perm], flow, solver, 1, sp.cuts)
    assert float((q2 - q1[perm]).abs().max()) <= 1e-14 * float(q1.abs().max())
    rbar = torch.randn(q.shape, generator=torch.Generator().manual_seed(6), dtype=O.DT)
    qb, xb, ab = O.residual_vjp(blocks, q, flow, solver, rbar)
    qbs, xbs, abs_ = O.residual_vjp(sblocks, q[perm], flow, solver, rbar[perm], sp.cuts)
    assert float((qbs - qb[perm]).abs().max()) <= 1e-12 * float(qb.abs().max())
    assert abs(float(ab) - float(abs_)) <= 1e-12 * abs(float(ab))


def _l_layout(scale):
    """The four-block C-grid layout (synth.c_grid_l) at 1/scale size beside
    the whole C-grid it is cut from: (big problem, L problem, perm, mask of
    the L cells whose stencil stays away from the two sides that face the
    part left out: the top rows of the first block, the imin columns of the
    upper block, and the corner of the second block under them)."""
    ni, nj, h = 448 // scale, 160 // scale, 64 // scale
    ib = [0, 256 // scale, 384 // scale, ni]
    fl = synth.flow_airfoil()
    fl.alpha0 = 0.03
    big = synth.Problem("big", [synth.Block(ni, nj, 1, synth.c_grid(ni, nj),
                                            (synth.FARFIELD, synth.FARFIELD, synth.WAKECUT,
                                             synth.FARFIELD), ni // 4, 0)], fl, synth.Solver(), 0, 3)
    blocks, cuts = synth.c_grid_l(1, scale)
    lp = synth.Problem("l", blocks, fl, synth.Solver(), 0, 3, cuts=cuts)
    ns = 3
    rects = [(ib[0], ib[1], 0, h), (ib[1], ib[2], 0, h), (ib[2], ni, 0, h), (ib[1], ni, h, nj)]
    perm = np.concatenate([synth._cell_perm(0, ns, nj, ni, j0, j1, i0, i1)
                           for i0, i1, j0, j1 in rects])
    masks = []
    for k, (i0, i1, j0, j1) in enumerate(rects):
        m = torch.ones(ns, 4, j1 - j0, i1 - i0, dtype=torch.bool)
        if k == 0:
            m[:, :, -3:, :] = False
        if k == 1:
            m[:, :, -3:, :3] = False
        if k == 3:
            m[:, :, :, :3] = False
        masks.append(m.reshape(-1))
    return big, lp, torch.as_tensor(perm), torch.cat(masks)


def test_four_block_c_grid_layout_equals_the_whole_grid_away_from_its_cut_off_sides():
    """The layout of the four-block airfoil configuration at 1/8 size
    (bottom layer 32 | 16 | 8 columns of 8 rows, 24 x 12 above the last
    two): every cell whose stencil does not reach the two far-field sides
    that face the part of the C-grid left out has the whole grid's
    residual, and the wall loads (all on the bottom layer) are the whole
    grid's.  The wake is glued over two segments of the first block's jmin
    (to the third block and to the end of the second), whose remaining
    cells are wall."""
    big, lp, perm, mask = _l_layout(8)
    assert [b.bc[2] for b in lp.blocks] == [synth.CUT_WALL, synth.CUT_WALL, synth.CUT, synth.CUT]
    bb, flow, solver = O.from_synth(big)
    lb, _, _ = O.from_synth(lp)
    q = torch.as_tensor(synth.initial_state(big))
    r = O.residual_all(bb, q, flow, solver)
    rl = O.residual_all(lb, q[perm], flow, solver, lp.cuts)
    err = (rl - r[perm]).abs()
    assert float(err[mask].max()) <= 1e-13 * float(r.abs().max())
    assert float(err[~mask].max()) > 1e-8 * float(r.abs().max())     # the cut-off sides matter
    cf = torch.cat([c.reshape(-1) for c in O.forces(bb, q, flow, solver)])
    cfl = torch.cat([c.reshape(-1) for c in O.forces(lb, q[perm], flow, solver, cuts=lp.cuts)])
    assert float((cf - cfl).abs().max()) <= 1e-13 * float(cf.abs().max())


def test_partly_glued_side_rules_and_validation():
    """Cells of a partly glued side that no segment covers follow the rest
    kind (the far-field rest: free stream ghosts; a wall rest: mirrored
    cells, and the jmin wall faces carry loads); segments of a partly glued
    side must not overlap but need not cover it; a fully glued side still
    must be covered."""
    p = synth.make_problem("cyl_tiny")
    sp, _ = synth.split_problem(p, 1, 2)
    inner, outer = sp.blocks
    # the outer piece's jmin glued only over its first half; the inner's
    # jmax: far field beyond the segment
    h = inner.ni // 2
    blocks = [synth.Block(inner.ni, inner.nj, inner.n_harm, inner.xy,
                          (inner.bc[0], inner.bc[1], inner.bc[2], synth.CUT_FARFIELD), 0, 0),
              synth.Block(outer.ni, outer.nj, outer.n_harm, outer.xy,
                          (outer.bc[0], outer.bc[1], synth.CUT_WALL, outer.bc[3]), 0, 0)]
    cuts = [(0, 3, 0, 1, 2, 0, h, 0)]
    ob, flow, solver = O.from_synth(synth.Problem("pg", blocks, p.flow, p.solver, 0, 1, cuts=cuts))
    P = O.cut_partners(ob, cuts)
    ws = [O.primitives(torch.as_tensor(synth.initial_state(synth.Problem("s", [b], p.flow, p.solver, 0, 1 + k)))
                       .reshape(b.ns, 4, b.nj, b.ni), flow.gamma) for k, b in enumerate(blocks)]
    winfs = [O.freestream_prim(flow, b.ns) for b in ob]
    we = O.extend_all(ob, ws, winfs, P)
    ni, nj = inner.ni, inner.nj
    for i in range(ni):
        for k in range(2):
            g = we[0][:, :, nj + 2 + k, i + 2]
            if i < h:
                assert torch.equal(g, ws[1][:, :, k, i])                      # glued
            else:
                assert torch.equal(g, winfs[0])                             # far-field rest
            g1 = we[1][:, :, 1 - k, i + 2]
            if i < h:
                assert torch.equal(g1, ws[0][:, :, nj - 1 - k, i])
            else:
                assert torch.equal(g1, O.mirror_prim(ws[1][:, :, k:k + 1, i:i + 1])[..., 0, 0])
    mask = O.wall_face_mask(ob[1], O.cut_ghost_centres(ob, P, [O.metrics(b.xy)[3] for b in ob], 1))
    assert mask.tolist() == [i >= h for i in range(ni)]
    O.cut_partners(ob, [])                                   # partly glued: may be uncovered
    with pytest.raises(ValueError):                          # overlap
        O.cut_partners(ob, cuts + [(0, 3, h - 1, 1, 2, h - 1, 2, 0)])
    full = [synth.Block(b.ni, b.nj, b.n_harm, b.xy, tuple(synth.CUT if k in (synth.CUT_WALL, synth.CUT_FARFIELD)
                                                         else k for k in b.bc), 0, 0) for b in blocks]
    fb, _, _ = O.from_synth(synth.Problem("f", full, p.flow, p.solver, 0, 1))
    with pytest.raises(ValueError):                          # a CUT side half covered
        O.cut_partners(fb, cuts)
