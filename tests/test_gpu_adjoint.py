"""GPU parity of the hand-written reverse-mode residual kernels: the
transposed-Jacobian products of R* with respect to the state, the node
coordinates and the mean incidence, against the FP64 oracle's reverse mode
(element by element) and against central finite differences of the GPU
residual itself; Hicks-Henne design gradients on the 256x128 airfoil."""
import numpy as np
import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("name", ["cyl_tiny", "naca_tiny", "batch_tiny"])
@pytest.mark.parametrize("batched", [0, 1])
def test_adjoint_matches_oracle(name, batched):
    _say("adjoint", name, "batched", batched)
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.02
    blocks, flow, solver = O.from_synth(p)
    q = torch.as_tensor(synth.initial_state(p))
    rbar = torch.randn(q.shape, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    qref, xyref, aref = O.residual_vjp(blocks, q, flow, solver, rbar)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=batched)
    qb = torch.empty_like(q, device=DEV)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    g.residual_adjoint(q.to(DEV), rbar.to(DEV), qb, xyb, ab)
    torch.cuda.synchronize()
    qb = qb.cpu()
    xyr = torch.cat([x.reshape(-1) for x in xyref])
    _say("  qbar rel", _rel(qb, qref), "xybar rel", _rel(xyb.cpu(), xyr),
         "alpha", float(ab), float(aref))
    assert _rel(qb, qref) <= 1e-11
    assert float((qb - qref).abs().max()) <= 1e-10 * float(qref.abs().max())
    assert _rel(xyb.cpu(), xyr) <= 1e-11
    assert abs(float(ab) - float(aref)) <= 1e-11 * abs(float(aref))


def test_adjoint_dot_product_with_gpu_differences():
    """<rbar, (R(q+hv) - R(q-hv)) / 2h> = <J^T rbar, v> using only the GPU."""
    p = synth.make_problem("naca_tiny")
    q = torch.as_tensor(synth.initial_state(p)).to(DEV)
    gen = torch.Generator().manual_seed(11)
    rbar = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV)
    v = (torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV) * q.abs() * 1e-2)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    qb = g.residual_adjoint(q, rbar)
    h = 1e-6
    fd = float((rbar * (g.residual(q + h * v) - g.residual(q - h * v))).sum()) / (2 * h)
    ad = float((qb * v).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_design_gradient_hicks_henne():
    """Adjoint of r^T R* with respect to the 64 Hicks-Henne amplitudes
    (beta_bar = (dXY/dbeta)^T xybar) and the inflow angle on the 256x128
    N_H = 2 airfoil: element-wise against the oracle's reverse mode, and
    against central differences of the GPU residual on re-built metrics.
    The residual is only piecewise smooth (the modulus of the convective Roe
    eigenvalues, Harten's switch on the acoustic ones): with h = 1e-6 the
    difference along bump 31 crosses such a kink and is off by 3e-5
    relative, while h = 1e-7 stays on one side (the oracle's own difference
    there agrees with its reverse mode to 3e-8)."""
    p = synth.make_problem("naca256x128_hh64")
    beta, dxy = p.design["beta"], p.design["dxy"]
    blocks, flow, solver = O.from_synth(p)
    qh = torch.as_tensor(synth.initial_state(p))
    q = qh.to(DEV)
    rbh = torch.randn(qh.shape, generator=torch.Generator().manual_seed(5), dtype=torch.float64)
    rbar = rbh.to(DEV)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    qb = g.residual_adjoint(q, rbar, None, xyb, ab)
    torch.cuda.synchronize()
    qref, xyref, aref = O.residual_vjp(blocks, qh, flow, solver, rbh)
    assert _rel(qb.cpu(), qref) <= 1e-11
    assert _rel(xyb.cpu(), xyref[0].reshape(-1)) <= 1e-11
    assert abs(float(ab) - float(aref)) <= 1e-11 * abs(float(aref))
    D = torch.as_tensor(dxy.reshape(len(beta), -1)).to(DEV)
    bbar = (D @ xyb).cpu()
    xy0 = torch.as_tensor(p.blocks[0].xy.reshape(-1)).to(DEV)

    def obj():
        return float((rbar * g.residual(q)).sum())

    def cd(set_fn, h):
        set_fn(h)
        fp = obj()
        set_fn(-h)
        fm = obj()
        return (fp - fm) / (2 * h)

    h = 1e-7
    for k in (0, 15, 31, 47, 63):
        fd = cd(lambda e: g.set_xy(xy0 + e * D[k]), h)
        _say("  beta", k, fd, float(bbar[k]))
        assert abs(fd - float(bbar[k])) <= 1e-6 * max(abs(fd), 1e-3 * float(bbar.abs().max()))
    g.set_xy(xy0)
    fd = cd(lambda e: g.set_alpha0(p.flow.alpha0 + e), h)
    g.set_alpha0(p.flow.alpha0)
    _say("  alpha0", fd, float(ab))
    assert abs(fd - float(ab)) <= 1e-6 * abs(fd)


def test_adjoint_large_block_against_gpu_differences():
    """A block of more than 65,536 cells takes the per-cell fold (smaller
    blocks fold one thread per cell and snapshot): the dot-product identity
    against central differences of the GPU residual in the state, the node
    coordinates and the incidence on the 1024x512 N_H = 4 airfoil."""
    p = synth.make_problem("naca1024x512_nh4")
    assert p.blocks[0].ni * p.blocks[0].nj >= 65536
    q = torch.as_tensor(synth.initial_state(p)).to(DEV)
    gen = torch.Generator().manual_seed(13)
    rbar = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=DEV)
    ab = torch.empty(1, dtype=torch.float64, device=DEV)
    qb = g.residual_adjoint(q, rbar, None, xyb, ab)

    def obj(qq):
        return float((rbar * g.residual(qq)).sum())

    v = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(DEV) * q.abs() * 1e-2
    h = 1e-6
    fd = (obj(q + h * v) - obj(q - h * v)) / (2 * h)
    ad = float((qb * v).sum())
    _say("  large state", fd, ad)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # a smooth deformation of the node coordinates (a random one is a poor
    # direction for differences of this piecewise-smooth operator).  With the
    # random rbar the difference is limited by truncation above displacements
    # of about 1e-7 (the first cells at the wall are thin) and by the rounding
    # of the 4.7e6-term sum below; 1e-8 displacements reach 2e-5 (the same
    # difference on the 256x128 grid, whose reverse products match the
    # oracle to 1e-11, reaches 1e-6 at best), hence the 1e-4 bound
    xy0 = torch.as_tensor(p.blocks[0].xy.reshape(-1)).to(DEV)
    nn = xy0.numel() // 2
    X, Y = xy0[:nn], xy0[nn:]
    dx = torch.cat([1e-4 * torch.sin(0.5 * X) * torch.cos(0.5 * Y),
                    1e-4 * torch.cos(0.3 * X) * torch.sin(0.7 * Y)])
    hx = 1e-4
    g.set_xy(xy0 + hx * dx)
    fp = obj(q)
    g.set_xy(xy0 - hx * dx)
    fm = obj(q)
    g.set_xy(xy0)
    fd = (fp - fm) / (2 * hx)
    ad = float((xyb * dx).sum())
    _say("  large coordinates", fd, ad)
    assert abs(fd - ad) <= 1e-4 * abs(ad), (fd, ad)
    # incidence: rotating the free stream moves the normal velocity of the
    # outer faces through zero, a kink of the Roe dissipation |q_n| (the
    # difference is -2.676, -2.579, -2.610, -2.6068 at h = 1e-4 .. 1e-7 against
    # the adjoint's -2.6067), so h = 1e-7 as for the design gradient, and the
    # bound allows the kinks still crossed at that h
    ha = 1e-7
    g.set_alpha0(p.flow.alpha0 + ha)
    fp = obj(q)
    g.set_alpha0(p.flow.alpha0 - ha)
    fm = obj(q)
    g.set_alpha0(p.flow.alpha0)
    fd = (fp - fm) / (2 * ha)
    _say("  large alpha0", fd, float(ab))
    assert abs(fd - float(ab)) <= 1e-4 * abs(fd), (fd, float(ab))
    g.close()


@pytest.mark.parametrize("name", ["cyl_tiny", "naca_tiny"])
def test_adjoint_iteration_stage_by_stage(name):
    """Two adjoint iterations lam <- lam0 - alpha_k (dtau/V)(J^T lam + gq)
    with the frozen local steps, against the same recursion on the oracle's
    reverse products (the first-stage norms too).  The iteration fills the
    ghost-extended copy of its fixed state once per call: a residual adjoint
    at another state run just before it, and a second iteration call after
    it, must not change its result (bit for bit against a fresh grid)."""
    p = synth.make_problem(name)
    p.flow.alpha0 = 0.02
    blocks, flow, solver = O.from_synth(p)
    q = torch.as_tensor(synth.initial_state(p))
    gen = torch.Generator().manual_seed(21)
    gq = torch.randn(q.shape, generator=gen, dtype=torch.float64)
    lam0 = 1e-2 * torch.randn(q.shape, generator=gen, dtype=torch.float64)
    q2 = q * (1.0 + 1e-2 * torch.randn(q.shape, generator=gen, dtype=torch.float64))
    g = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=0, batched=1)
    lg = lam0.to(DEV)
    norms = torch.zeros(2, dtype=torch.float64, device=DEV)
    g.residual_adjoint(q2.to(DEV), gq.to(DEV))                 # another state first
    g.adjoint_iterate(q.to(DEV), lg, gq.to(DEV), 2, norms)
    torch.cuda.synchronize()
    vols = [O.metrics(b.xy)[2] for b in blocks]
    dtv = O.join([(O.local_dt(b, qb, flow, solver) / V)[:, None].expand(-1, 4, -1, -1)
                  for b, qb, V in zip(blocks, O.split(blocks, q), vols)])
    lam, ref_norms = lam0.clone(), []
    for _ in range(2):
        base = lam.clone()
        for k, a in enumerate(solver.rk_alpha):
            r = O.residual_vjp(blocks, q, flow, solver, lam, p.cuts)[0] + gq
            if k == 0:
                s = sum(float(((rb / V) ** 2).sum()) for rb, V in zip(O.split(blocks, r), vols))
                ref_norms.append((s / q.numel()) ** 0.5)
            lam = base - a * dtv * r
    err = _rel(lg.cpu(), lam)
    _say("  lambda rel", err, "norms", norms.cpu().tolist(), ref_norms)
    assert err <= 1e-11
    for a, b in zip(norms.cpu().tolist(), ref_norms):
        assert abs(a - b) <= 1e-11 * b
    # the same two iterations on a fresh grid, and a second call on this one
    g2 = hb.Grid(p.blocks, p.flow, p.solver, cuts=p.cuts, precision=0, batched=1)
    lf = lam0.to(DEV)
    g2.adjoint_iterate(q.to(DEV), lf, gq.to(DEV), 2)
    lr = lam0.to(DEV)
    g.adjoint_iterate(q.to(DEV), lr, gq.to(DEV), 2)
    torch.cuda.synchronize()
    assert torch.equal(lf, lg) and torch.equal(lr, lg)
    g.close()
    g2.close()
