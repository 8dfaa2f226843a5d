"""The secondary legs of bench.py (finite box, toy-model sweep) run as the
default benchmark runs them, so that a failure there shows up in the test
suite and not only in a benchmark line."""
import os
import sys

import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_finite_and_toy_legs():
    import math
    import bench
    note("bench legs: finite box")
    f = bench.run_finite(3)
    note(f"  {f}")
    for k in ("finite_f32_ms_per_step", "finite_f64_ms_per_step", "periodic_f32_ms_per_step"):
        assert f[k] > 0.0
    assert abs(f["finite_f32_energy_change"]) < 1e-3 * 30.0
    note("bench legs: toy sweep")
    t = bench.run_toy(oracle_sample=False)
    for sch in ("ehrenfest", "cp"):
        r = t[sch]
        note(f"  {sch}: {r['kernel_ms']} ms, {r['rk4_steps_per_s']:.3e} steps/s")
        assert r["kernel_ms"] > 0.0 and r["n_traj"] > 0
        assert all(math.isfinite(x) for x in r["d_R"])
