"""Pin the oracle's reverse-mode products (automatic differentiation of the
FP64 residual) with central finite differences: the dot-product identity
<rbar, J v> = <J^T rbar, v> for random directions in the state, the node
coordinates and the incidence (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import hb_oracle as O
from paper_1304_7654_amd import synth

DT = torch.float64


@pytest.mark.parametrize("name", ["naca_tiny", "cyl_tiny"])
def test_vjp_matches_central_differences(name):
    p = synth.make_problem(name)
    blocks, flow, solver = O.from_synth(p)
    flow.alpha0 = 0.02
    q = torch.as_tensor(synth.initial_state(p))
    gen = torch.Generator().manual_seed(7)
    rbar = torch.randn(q.shape, generator=gen, dtype=DT)
    qbar, xybars, abar = O.residual_vjp(blocks, q, flow, solver, rbar)

    def obj(qq=q, xys=None, a0=None):
        return float((O.residual_with(blocks, qq, flow, solver, xys, a0) * rbar).sum())

    # state direction
    v = torch.randn(q.shape, generator=gen, dtype=DT) * q.abs() * 1e-2
    h = 1e-6
    fd = (obj(q + h * v) - obj(q - h * v)) / (2 * h)
    ad = float((qbar * v).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # node-coordinate direction (smooth, small)
    dx = [torch.randn(b.xy.shape, generator=gen, dtype=DT) * 1e-3 for b in blocks]
    hx = 1e-5
    fd = (obj(xys=[b.xy + hx * d for b, d in zip(blocks, dx)])
          - obj(xys=[b.xy - hx * d for b, d in zip(blocks, dx)])) / (2 * hx)
    ad = sum(float((g * d).sum()) for g, d in zip(xybars, dx))
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # incidence
    ha = 1e-6
    fd = (obj(a0=flow.alpha0 + ha) - obj(a0=flow.alpha0 - ha)) / (2 * ha)
    assert abs(fd - float(abar)) <= 1e-6 * abs(float(abar)), (fd, float(abar))


@pytest.mark.parametrize("name", ["naca_tiny", "cyl_tiny"])
def test_forces_vjp_matches_central_differences(name):
    p = synth.make_problem(name)
    blocks, flow, solver = O.from_synth(p)
    flow.alpha0 = 0.02
    q = torch.as_tensor(synth.initial_state(p))
    gen = torch.Generator().manual_seed(8)
    n_cf = sum(b.ns for b in blocks) * 3
    cfbar = torch.randn(n_cf, generator=gen, dtype=DT)
    qbar, xybars, abar = O.forces_vjp(blocks, q, flow, solver, cfbar)
    assert float(qbar.abs().max()) > 0 and float(abar) != 0.0

    def obj(qq=q, xys=None, a0=None):
        return float((O.forces_with(blocks, qq, flow, solver, xys, a0) * cfbar).sum())

    v = torch.randn(q.shape, generator=gen, dtype=DT) * q.abs() * 1e-2
    h = 1e-6
    fd = (obj(q + h * v) - obj(q - h * v)) / (2 * h)
    ad = float((qbar * v).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    dx = [torch.randn(b.xy.shape, generator=gen, dtype=DT) * 1e-3 for b in blocks]
    hx = 1e-5
    fd = (obj(xys=[b.xy + hx * d for b, d in zip(blocks, dx)])
          - obj(xys=[b.xy - hx * d for b, d in zip(blocks, dx)])) / (2 * hx)
    ad = sum(float((g * d).sum()) for g, d in zip(xybars, dx))
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    ha = 1e-6
    fd = (obj(a0=flow.alpha0 + ha) - obj(a0=flow.alpha0 - ha)) / (2 * ha)
    assert abs(fd - float(abar)) <= 1e-6 * abs(float(abar)), (fd, float(abar))
