"""The oracle's operation counter counts what it claims (CPU)."""
import torch

from oracle import hb_opcount as C
from oracle import hb_oracle as O
from paper_1304_7654_amd import synth


def test_counter_on_known_expressions():
    a = torch.rand(7, 5, dtype=torch.float64)
    b = torch.rand(7, 5, dtype=torch.float64)
    _, c = C.count(lambda: a * b + torch.sqrt(a) / b)
    assert c.total == 4 * 35
    m = torch.rand(6, 4, dtype=torch.float64)
    n = torch.rand(4, 3, dtype=torch.float64)
    _, c = C.count(lambda: m @ n)
    assert c.total == 2 * 6 * 3 * 4
    _, c = C.count(lambda: a.sum(-1))
    assert c.total == 35 - 7
    # integer and index work is not counted
    _, c = C.count(lambda: (torch.arange(10) * 3, a[:, 0].clone(), torch.stack([a, b])))
    assert c.total == 0


def test_residual_ops_per_cell_snapshot_are_size_independent():
    """The per-unit count converges with block size (boundary work is a
    perimeter term) and is of the order of the face arithmetic: two faces
    per cell, each a MUSCL reconstruction, a Roe flux and a viscous flux."""
    per = []
    for n in (16, 32):
        p = synth.make_problem("cyl_tiny")
        p.blocks = [synth.o_block(2 * n, n, 1)]
        blocks, flow, solver = O.from_synth(p)
        q = torch.as_tensor(synth.initial_state(p))
        per.append(C.ops_per_unit(blocks, q, flow, solver))
    r0, r1 = per[0]["residual_per_cell_snapshot"], per[1]["residual_per_cell_snapshot"]
    assert abs(r0 - r1) < 0.1 * r1
    assert 300 < r1 < 3000
    assert per[1]["per_unit"] > r1
