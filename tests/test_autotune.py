"""Autotuner objectives (CPU): how phase times combine into what is minimised."""
import pytest

from paper_1806_05713_amd import autotune


def test_objectives_from_phase_times():
    t = autotune.timings({"cells": 20.0, "neigh": 80.0, "force": 50.0, "other": 6.0})
    assert t["build_us"] == pytest.approx(100.0)
    assert t["force_us"] == pytest.approx(50.0)
    assert t["step_us"] == pytest.approx(156.0)
    # an integrator step: every step's forces, a tenth of a rebuild
    assert t["nve_us"] == pytest.approx(56.0 + 100.0 / autotune.NVE_REBUILD_EVERY)


def test_nve_objective_prefers_cheaper_forces():
    fast_build = autotune.timings({"cells": 20.0, "neigh": 60.0, "force": 60.0, "other": 6.0})
    fast_force = autotune.timings({"cells": 20.0, "neigh": 90.0, "force": 50.0, "other": 6.0})
    assert fast_build["step_us"] < fast_force["step_us"]
    assert fast_force["nve_us"] < fast_build["nve_us"]
