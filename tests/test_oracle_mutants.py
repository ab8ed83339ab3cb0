"""Planted mistakes: each mutant is a copy of the oracle's C source with one
plausible error (a dropped term, a wrong sign, index or exponent, a transposed
operand, a missing stencil cell, ...).  It is compiled on the CPU into a
temporary library and run through the pins of test_oracle_pins; every mutant
must fail at least one pin.  This shows the pins bind the oracle, not only
that the oracle passes them."""
import os
import tempfile

import numpy as np
import pytest

from oracle import ljref
from tests import test_oracle_pins as pins
from paper_1806_05713_amd import synth

MUTANTS = {
    "i-force-sign": ("fi[0] -= fs * t[0];", "fi[0] += fs * t[0];"),
    "j-force-sign (Alg.1 as printed)": ("force[3 * (int64_t)j + 1] += fs * t[1];",
                                        "force[3 * (int64_t)j + 1] -= fs * t[1];"),
    "dropped-shift": ("ksum_add(&E, 4.0 * eps * sr6 * (sr6 - 1.0) - vc);\n            ksum_add(&W, fs * r2);\n            ++count;",
                      "ksum_add(&E, 4.0 * eps * sr6 * (sr6 - 1.0));\n            ksum_add(&W, fs * r2);\n            ++count;"),
    "r^4-not-r^6": ("const double sr6 = sr2 * sr2 * sr2;\n            const double fs = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;\n            /* t points",
                    "const double sr6 = sr2 * sr2;\n            const double fs = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;\n            /* t points"),
    "virial-missing-r2": ("ksum_add(&W, fs * r2);\n            ++count;", "ksum_add(&W, fs);\n            ++count;"),
    "min-image-sign": ("        t -= L;", "        t += L;"),
    "transposed-z": ("t[2] = min_image(qj[2] - qi[2], box[2]);", "t[2] = min_image(qi[2] - qj[2], box[2]);"),
    "r2-wrong-index": ("(t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]", "(t[0] * t[0] + t[1] * t[1]) + t[1] * t[1]"),
    "self-pair": ("if (j <= i) continue;", "if (j < i) continue;"),
    "force-constant-48": ("const double fs = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;\n            /* t points",
                          "const double fs = 48.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;\n            /* t points"),
    "stencil-missing-dx": ("for (int dx = -1; dx <= 1; ++dx)", "for (int dx = 0; dx <= 1; ++dx)"),
    "cells-smaller-than-rs": ("int nc = (int)floor(box[d] / rs);\n        while (nc > 1 && box[d] / nc < rs * (1.0 + 1e-12)) --nc;",
                              "int nc = (int)floor(box[d] / rs) + 1;"),
    "cutoff-at-rs": ("const double rc2 = rc * rc;\n    const double sig2 = sigma * sigma;\n    const double vc",
                     "const double rc2 = (rc + 0.3) * (rc + 0.3);\n    const double sig2 = sigma * sigma;\n    const double vc"),
    "full-kick": ("for (int64_t k = 0; k < 3 * n; ++k) vel[k] += 0.5 * dt * force[k];\n            for (int64_t i",
                  "for (int64_t k = 0; k < 3 * n; ++k) vel[k] += dt * force[k];\n            for (int64_t i"),
    "no-wrap-drift": ("x = x - box[d] * floor(x / box[d]);", "x = x - box[d] * floor(x / box[d] - 0.5);"),
}


def battery(O):
    """Run the pins on oracle O; return the names of those that fail."""
    failed = []

    def run(name, fn, *args):
        try:
            with np.errstate(all="ignore"):
                fn(O, *args)
        except Exception:  # an assertion, a NaN comparison, a status error
            failed.append(name)

    run("closed-forms", pins.test_two_particle_closed_forms, 1.0, 1.0, 0, False)
    run("closed-forms-face", pins.test_two_particle_closed_forms, 0.7, 1.3, 2, True)
    run("gradient", pins.test_force_is_minus_gradient, 1)
    run("virial", pins.test_virial_is_minus_scaling_derivative)
    run("net-force", pins.test_newton_third_law_zero_net_force, lambda: synth.small_fcc(6, 1.0, 0.1, 2))
    run("shells", pins.test_perfect_fcc_neighbor_shells, 1.0)
    run("lattice-sum", pins.test_perfect_fcc_lattice_sum, 0.85, 2.5, 5)
    for name, maker, _ in pins.CASES:
        run("definition-" + name, pins.test_cell_list_equals_definition, name, maker, None)
    run("nve", pins.test_nve_energy_conservation)
    run("nve-reverse", pins.test_nve_time_reversible)
    return failed


def test_true_oracle_passes_battery(oracle):
    assert battery(oracle) == []


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(ljref.SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "ljref.c")
        with open(c, "w") as f:
            f.write(mutated)
        with open(os.path.join(d, "ljref.h"), "w") as f:
            f.write(open(os.path.join(ljref.HERE, "ljref.h")).read())
        so = ljref.build(src=c, out=os.path.join(d, "libljref_mut.so"))
        failed = battery(ljref.Oracle(so))
    assert failed, f"mutant {name} passed every pin"
