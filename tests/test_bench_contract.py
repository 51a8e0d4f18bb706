"""The benchmark's host-side contract, without a GPU: the one-GPU guard, the
roofline's per-unit slot counts (itemised necessary operations, priced with
the measured instruction costs), the count of moved estimates, and the probe
library's kernels matching the benchmark's tables."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_slot_counts_are_the_sums_of_their_items():
    for form, stages in bench.SLOT_ITEMS.items():
        for stage, items in stages.items():
            assert bench.SLOTS[form][stage] == pytest.approx(sum(items.values()), abs=1e-9)
    # the FP64 likelihood: 9.3 slots per (cell, e point, knot): x 1, rsqrt 4,
    # cube 2, D and M 2 (sqrt(W) carried by the profile), quadratic form 0.3
    assert bench.SLOTS["fp64"]["fit"] == pytest.approx(9.3)
    # v_rsq_f64 is priced at 4 slots wherever the FP64 form takes a rsqrt;
    # FP32 transcendentals at 1 in the mixed form
    for stage in ("model", "extract", "fit"):
        assert bench.SLOT_ITEMS["fp64"][stage]["rsqrt"] == 4
        assert bench.SLOT_ITEMS["mixed"][stage]["rsqrt"] == 1
    assert bench.SLOT_ITEMS["fp64"]["model"]["sin + cos"] == 8
    assert bench.SLOT_ITEMS["mixed"]["model"]["sin + cos"] == 2
    # the mixed form needs no more work per unit than the FP64 form
    for stage in ("model", "extract", "fit"):
        assert bench.SLOTS["mixed"][stage] <= bench.SLOTS["fp64"][stage]


def test_roofline_peak_and_fraction_formula():
    assert bench.SLOT_PEAK == pytest.approx(256 * 64 * 2.4e9)
    # the headline stage at a measured config-1 time: 9.3 slots x 295,955
    # cells x 6,333 points x 20 knots in 12.0 ms
    units = 295955 * 6333 * 20
    frac = bench.SLOTS["fp64"]["fit"] * units / 12.0e-3 / bench.SLOT_PEAK
    assert 0.7 < frac < 0.8


def test_sources_whose_estimate_moved():
    # e1 differences of three sources, then their e2 differences
    de = np.array([0.0, 2e-3, 0.0, 0.0, 0.0, -5e-3])
    assert bench._sources_de_above(de) == 2
    assert bench._sources_de_above(np.zeros(8)) == 0
    assert bench._sources_de_above(de, tol=3e-3) == 1


def test_probe_library_matches_the_benchmark_tables():
    from paper_2203_14071_amd import build
    if not os.path.exists(build.PROBE_LIB):
        pytest.skip("probe library not built")
    L = ctypes.CDLL(build.PROBE_LIB)
    assert L.valu_probe_count() == len(bench.PROBES)
    assert L.mix_probe_count() == len(bench.MIX_PROBES)
    # each kernel-mix probe bounds one (form, stage) roofline
    keys = [p[1] for p in bench.MIX_PROBES]
    assert len(set(keys)) == len(keys)
    for form, stage in keys:
        assert stage in bench.SLOTS[form]
