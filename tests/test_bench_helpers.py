"""Host-side helpers of bench.py that name the measured kernels and count
their algorithmic VALU slots (no GPU: the names must match what rocprofv3
prints for the kernels the plan launches, and the slot counts the plan's
formulation)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sweep_kernel_names_follow_the_plan():
    stored = {"edge_state": 1}
    assert bench.sweep_kernel_name("mixed", stored) == "gabp::k_sweep<float, double, double, 0, 0, 0, false, 0>"
    chunked = {"edge_state": 2, "stateless_depth": 3, "series_reciprocal": 3, "tile_chunk": 2}
    assert bench.sweep_kernel_name("mixed", chunked) == "gabp::k_sweep_chunk<float, double, double, 0, 3, 3, 2>"
    assert bench.sweep_kernel_name("fp32", chunked) == "gabp::k_sweep_chunk<float, float, float, 0, 3, 3, 2>"
    tiles = dict(chunked, tile_chunk=1, stateless_depth=2, series_reciprocal=1)
    assert bench.sweep_kernel_name("fp32", tiles) == "gabp::k_sweep<float, float, float, 0, 0, 2, false, 1>"
    assert bench.sweep_label(chunked, "stateless").startswith("k_sweep_chunk (stateless, 2 x 2 tile chunks")
    assert bench.sweep_label(tiles, "stateless", ", FP32") == "k_sweep (stateless, K' materialised, FP32)"


def test_kernel_base_name_drops_the_return_type():
    assert bench.kernel_base_name("void gabp::k_status(int)") == "gabp::k_status(int)"
    assert bench.kernel_base_name("gabp::k_stage(float)") == "gabp::k_stage(float)"


def test_recompute_slots_follow_the_k_formulation():
    # K' from the plain Gram: distance 3, scale 1, exp2 4, + lambda^2 1; from
    # augmented rows: clamp 1, exp2 4, + lambda^2 1
    assert bench.recompute_slots({"recompute_aug": 0}) == 9
    assert bench.recompute_slots({"recompute_aug": 1}) == 6
    assert bench.recompute_slots({}) == 9
    # series form 3 at three levels: a^2 1, middle level 4, top level 12
    assert bench.stateless_slots_per_pair(3, 3) == 17
