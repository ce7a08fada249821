"""CPU-side checks of the C ABI: the library loads, exports every function
the header declares, the ctypes structures match the C layout, and
argument validation fails before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1304_7654_amd import hb, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = hb.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hb.EXPORTS)


def test_struct_layout_matches_header():
    """Compile a tiny C program against include/hb.h with gcc and compare
    sizeof/offsetof with the ctypes mirrors of the binding."""
    prog = r'''
#include <stddef.h>
#include <stdio.h>
#include "hb.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(hb_block), sizeof(hb_cut), sizeof(hb_flow), sizeof(hb_solver));
  printf("%zu %zu %zu %zu\n", offsetof(hb_block, xy), offsetof(hb_block, bc),
         offsetof(hb_block, wake_ncells), offsetof(hb_block, body_id));
  printf("%zu %zu %zu %zu\n", offsetof(hb_solver, rk_alpha), offsetof(hb_solver, precision),
         offsetof(hb_solver, limiter_eps), offsetof(hb_solver, graph_iters));
  printf("%zu %zu %zu\n", sizeof(hb_tuning), offsetof(hb_tuning, tile_order),
         offsetof(hb_tuning, stage_ms));
  printf("%zu %zu\n", sizeof(hb_motion), offsetof(hb_motion, y_pivot));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    got = [int(x) for x in out]
    ref = [ctypes.sizeof(hb.c_block), ctypes.sizeof(hb.c_cut), ctypes.sizeof(hb.c_flow),
           ctypes.sizeof(hb.c_solver),
           hb.c_block.xy.offset, hb.c_block.bc.offset, hb.c_block.wake_ncells.offset,
           hb.c_block.body_id.offset,
           hb.c_solver.rk_alpha.offset, hb.c_solver.precision.offset,
           hb.c_solver.limiter_eps.offset, hb.c_solver.graph_iters.offset,
           ctypes.sizeof(hb.c_tuning), hb.c_tuning.tile_order.offset, hb.c_tuning.stage_ms.offset,
           ctypes.sizeof(hb.c_motion), hb.c_motion.y_pivot.offset]
    assert got == ref


def _try(blocks, flow=None, solver=None, cuts=()):
    p = synth.make_problem("cyl_tiny")
    with pytest.raises(hb.HBError) as e:
        hb.Grid(blocks, flow or p.flow, solver or p.solver, cuts)
    return e.value.code


def test_validation_rejects_before_device_work():
    p = synth.make_problem("cyl_tiny")
    b = p.blocks[0]
    assert _try([]) == hb.HB_ERR_ARG
    bad = synth.Block(b.ni, b.nj, 5, b.xy, b.bc)
    assert _try([bad]) == hb.HB_ERR_ARG                      # n_harm > 4
    bad = synth.Block(3, b.nj, 1, b.xy, b.bc)
    assert _try([bad]) == hb.HB_ERR_ARG                      # too small
    bad = synth.Block(b.ni, b.nj, 1, b.xy, (9, 9, 1, 2))
    assert _try([bad]) == hb.HB_ERR_ARG                      # unknown bc
    bad = synth.Block(b.ni, b.nj, 1, b.xy, (synth.PERIODIC, synth.FARFIELD, 1, 2))
    assert _try([bad]) == hb.HB_ERR_ARG                      # unpaired periodic
    bad = synth.Block(b.ni, b.nj, 1, b.xy, (3, 3, synth.WALL, synth.WAKECUT))
    assert _try([bad]) == hb.HB_ERR_ARG                      # wake cut not on jmin
    flipped = b.xy[:, :, ::-1].copy()                         # left-handed: negative areas
    bad = synth.Block(b.ni, b.nj, 1, flipped, b.bc)
    assert _try([bad]) == hb.HB_ERR_ARG
    b2 = synth.Block(b.ni, b.nj, 2, b.xy, b.bc, 0, 0)
    assert _try([b, b2]) == hb.HB_ERR_ARG                    # one body, two n_harm
    b3 = synth.Block(b.ni, b.nj, 1, b.xy, b.bc, 0, 2)
    assert _try([b, b3]) == hb.HB_ERR_ARG                    # body ids with a gap
    s = synth.Solver(precision=1, batched=0)
    assert _try([b], solver=s) == hb.HB_ERR_ARG              # FP32 bulk needs batched
    s = synth.Solver(cfl=-1.0)
    assert _try([b], solver=s) == hb.HB_ERR_ARG
    f = synth.Flow(mach=0.0, reynolds=100.0)
    assert _try([b], flow=f) == hb.HB_ERR_ARG
    cut = synth.Block(b.ni, b.nj, 1, b.xy, (3, 3, synth.CUT, 2))
    assert _try([cut]) == hb.HB_ERR_ARG                      # CUT side without a cut
    assert "n_harm" in hb.lib().hb_last_error().decode() or True
    # cuts are segments of sides: each HB_BC_CUT side must be covered by its
    # segments exactly once, inside the sides, with a reversed flag of 0 or 1
    sp, _ = synth.split_problem(p, 2, 1)
    a, sa, b2_, sb = sp.cuts[0][:4]
    side = sp.blocks[a].nj if sa < 2 else sp.blocks[a].ni
    others = list(sp.cuts[1:])
    for cuts in ([(a, sa, 0, b2_, sb, 0, side - 2, 0)] + others,          # side not covered
                 [(a, sa, 0, b2_, sb, 0, side, 0), (a, sa, 0, b2_, sb, 0, 2, 0)] + others,  # overlap
                 [(a, sa, 1, b2_, sb, 1, side, 0)] + others,              # leaves the side
                 [(a, sa, 0, b2_, sb, 0, side + 1, 0)] + others,
                 [(a, sa, -1, b2_, sb, 0, side, 0)] + others,
                 [(a, sa, 0, b2_, sb, 0, 0, 0)] + others,
                 [(a, sa, 0, b2_, sb, 0, side, 2)] + others):            # reversed must be 0 or 1
        with pytest.raises(hb.HBError) as e:
            hb.Grid(sp.blocks, sp.flow, sp.solver, cuts)
        assert e.value.code == hb.HB_ERR_ARG, cuts
    # partly glued sides (HB_BC_CUT_WALL / HB_BC_CUT_FARFIELD): segments may
    # leave cells uncovered but must not overlap; kinds above 7 are unknown
    pl = [synth.Block(x.ni, x.nj, x.n_harm, x.xy,
                      tuple(synth.CUT_WALL if k == synth.CUT else k for k in x.bc), 0, 0)
          for x in sp.blocks]
    part = [(a, sa, 0, b2_, sb, 0, side - 2, 0)] + others
    assert _try(pl, cuts=part) != hb.HB_ERR_ARG               # passes validation
    assert _try(pl, cuts=[(a, sa, 0, b2_, sb, 0, 3, 0), (a, sa, 2, b2_, sb, 2, 3, 0)] + others) \
        == hb.HB_ERR_ARG                                       # overlap
    odd = synth.Block(b.ni, b.nj, 1, b.xy, (3, 3, 8, 2))
    assert _try([odd]) == hb.HB_ERR_ARG


def test_binding_rejects_bad_tensors():
    import torch
    with pytest.raises(TypeError):
        hb._ptr(torch.zeros(4, dtype=torch.float32), 4, "q")
    with pytest.raises(TypeError):
        hb._ptr(torch.zeros(4, dtype=torch.float64), 4, "q")    # host tensor


def test_null_handles():
    L = hb.lib()
    assert L.hb_state_size(None) == -1
    assert L.hb_grid_destroy(None) == 0
    assert L.hb_residual(None, None, None, None) == hb.HB_ERR_ARG
    assert L.hb_get_status(None) == hb.HB_ERR_ARG
    m = hb.c_motion(0.1, 0.0, 0.2, 0.0, 0.0)
    assert L.hb_set_motion(None, ctypes.byref(m)) == hb.HB_ERR_ARG
    assert L.hb_prepare(None, hb.HB_PREPARE_TD) == hb.HB_ERR_ARG


def test_prepare_flags_match_header():
    """The hb_prepare bits of the binding are the header's."""
    src = open(os.path.join(ROOT, "include", "hb.h")).read()
    for name in ("HB_PREPARE_ADJOINT", "HB_PREPARE_ADJOINT_ITERATE", "HB_PREPARE_TD"):
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, src)
        assert m and int(m.group(1)) == getattr(hb, name), name


def test_committed_tuning_cache_matches_the_reader_format():
    """The library reads its tuning cache one entry per line with a fixed
    field order (hb_tune.cpp); every entry of the committed cache must be in
    that form, or a lookup silently misses and the autotuner runs again."""
    import json
    path = os.path.join(ROOT, "paper_1304_7654_amd", "tune_cache.json")
    text = open(path).read()
    entries = json.loads(text)
    pat = re.compile(r'^  "([^"]+)": \{"tile_i": (-?\d+), "wg_per_cu": (-?\d+), "xcd_order": (-?\d+), '
                     r'"tile_order": (-?\d+), "stage_ms": ([0-9.eE+-]+)\},?$')
    lines = [l for l in text.splitlines() if l not in ("{", "}")]
    assert len(lines) == len(entries) >= 1
    for l in lines:
        m = pat.match(l)
        assert m, l
        t = entries[m.group(1)]
        assert [t["tile_i"], t["wg_per_cu"], t["xcd_order"], t["tile_order"]] == \
            [int(m.group(k)) for k in range(2, 6)]


def test_size_limits_rejected_before_device_work():
    """More than 2^24 cells in a block is a bad argument, and so is a batched
    mode other than 0, 1 and 2; both are refused on the host.  (The state
    size is not limited: a batched grid of 4 GiB or more addresses its halo
    with 64-bit offsets.)"""
    p = synth.make_problem("cyl_tiny")
    n = 4097                                   # n * n > 2^24; the nodes are never read
    big = synth.Block(n, n, 0, np.zeros((2, n + 1, n + 1)), (synth.PERIODIC, synth.PERIODIC,
                                                              synth.WALL, synth.FARFIELD))
    assert _try([big]) == hb.HB_ERR_ARG
    for mode in (-1, 3):
        with pytest.raises(hb.HBError) as e:
            hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=mode)
        assert e.value.code == hb.HB_ERR_ARG
