"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the
counter-summary lookup, and that the committed summaries belong to the
current kernel source and the committed tuning (otherwise the benchmark
line reports no measured traffic)."""
import json
import os
import subprocess
import sys

import bench
from paper_1304_7654_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _committed_tuning(workload_blocks):
    cache = json.load(open(os.path.join(ROOT, "paper_1304_7654_amd", "tune_cache.json")))
    (key, t), = [(k, v) for k, v in cache.items() if "/blocks%d/prec1/" % workload_blocks in k]
    return t


def test_committed_summaries_match_kernel_and_tuning():
    t = _committed_tuning(32)
    assert bench.read_traffic(t, "batch32_mixed") is not None
    assert bench.read_profile_value(bench.profile_file("batch32_mixed", "sq_counters"),
                                    "valu_wave_instructions_per_launch", t, "batch32_mixed")
    t3 = _committed_tuning(1)
    assert bench.read_traffic(t3, "naca1024x512_nh4") is not None


def test_summary_lookup_is_keyed_by_workload_and_tuning():
    t = _committed_tuning(32)
    assert bench.read_traffic(t, "naca1024x512_nh4") is None          # another workload's file
    other = dict(t, tile_i=32 if t["tile_i"] == 16 else 16)
    assert bench.read_traffic(other, "batch32_mixed") is None        # another tuning


def test_plain_stage_bytes():
    p = synth.make_problem("batch32_mixed")
    fixed, moving = bench.plain_stage_bytes(p, False), bench.plain_stage_bytes(p, True)
    # at least Q in and out, E written once and read twice, both flux arrays out and in
    assert fixed > 8 * 4 * p.cell_snapshots * 2 * 5
    assert moving > fixed


def test_algorithmic_bytes_follow_the_unit_counts():
    """64 + 20/N_s B per unit for the FP32-shadow path and 88 + 40/N_s for
    FP64 stage states, summed over the blocks of the batch."""
    p = synth.make_problem("batch32_mixed")
    cs = p.cell_snapshots
    cells = sum(b.ni * b.nj for b in p.blocks)
    per_launch = bench.algorithmic_bytes_per_iteration(p) / 4
    assert abs(per_launch - (64 * cs + 20 * cells)) < 1e-6 * per_launch
    assert bench.design_bytes_per_iteration(p) / 4 - per_launch == 16 * cells
    plain = bench.plain_algorithmic_stage_bytes(p)
    assert abs(plain - (88 * cs + 40 * cells)) < 1e-6 * plain
    assert bench.plain_stage_bytes(p, False) > plain
