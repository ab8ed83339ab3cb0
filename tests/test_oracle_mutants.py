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
    "dropped-shift": ("double v = 4.0 * p->eps * sr6 * (sr6 - 1.0) - p->vc;",
                      "double v = 4.0 * p->eps * sr6 * (sr6 - 1.0);"),
    "r^4-not-r^6": ("const double sr6 = sr2 * sr2 * sr2;\n    double f",
                    "const double sr6 = sr2 * sr2;\n    double f"),
    "virial-missing-r2": ("ksum_add(&W, fs * r2);\n            ++count;", "ksum_add(&W, fs);\n            ++count;"),
    "min-image-sign": ("        t -= L;", "        t += L;"),
    "transposed-z": ("t[2] = min_image(qj[2] - qi[2], box[2]);", "t[2] = min_image(qi[2] - qj[2], box[2]);"),
    "r2-wrong-index": ("(t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]", "(t[0] * t[0] + t[1] * t[1]) + t[1] * t[1]"),
    "self-pair": ("if (j <= i) continue;", "if (j < i) continue;"),
    "force-constant-48": ("double f = 24.0 * p->eps", "double f = 48.0 * p->eps"),
    "stencil-missing-dx": ("for (int dx = -1; dx <= 1; ++dx)", "for (int dx = 0; dx <= 1; ++dx)"),
    "cells-smaller-than-rs": ("int nc = (int)floor(box[d] / rs);\n        while (nc > 1 && box[d] / nc < rs * (1.0 + 1e-12)) --nc;",
                              "int nc = (int)floor(box[d] / rs) + 1;"),
    "cutoff-at-rs": ("p->rc2 = rc * rc;", "p->rc2 = (rc + 0.3) * (rc + 0.3);"),
    "full-kick": ("for (int64_t k = 0; k < 3 * n; ++k) vel[k] += 0.5 * dt * force[k];\n            double dmax",
                  "for (int64_t k = 0; k < 3 * n; ++k) vel[k] += dt * force[k];\n            double dmax"),
    "no-wrap-drift": ("x = x - box[d] * floor(x / box[d]);", "x = x - box[d] * floor(x / box[d] - 0.5);"),
    # force-shifted truncation
    "fs-force-sign": ("f = f - p->fc / r;", "f = f + p->fc / r;"),
    "fs-energy-sign": ("v = v + (r - p->rc) * p->fc;", "v = v - (r - p->rc) * p->fc;"),
    "fs-no-linear-term": ("v = v + (r - p->rc) * p->fc;", "v = v + 0.0 * p->fc;"),
    "fs-constant-wrong-power": ("return 24.0 * eps * s6 * (2.0 * s6 - 1.0) / rc;",
                                "return 24.0 * eps * s6 * (2.0 * s6 - 1.0) / (rc * rc);"),
    # full list and sampler
    "full-list-energy-not-halved": ("*energy = 0.5 * ksum_get(&E);\n    *virial = 0.5",
                                    "*energy = ksum_get(&E);\n    *virial = 0.5"),
    "full-list-drops-lower-partners": (
        "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) fcol[fill[col[k]]++] = (int32_t)i;",
        "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) fcol[fill[col[k]]++] = col[k];"),
    "sample-rows-unsorted": ("while (b >= 0 && row[b] > v) {", "while (b >= 0 && row[b] > v && 0) {"),
    "sample-virial-not-halved": ("w[s] = 0.5 * ksum_get(&W);", "w[s] = ksum_get(&W);"),
    # displacement-triggered rebuild
    "trigger-at-skin-not-half": ("const double half_skin2 = (0.5 * skin) * (0.5 * skin);",
                                 "const double half_skin2 = skin * skin;"),
    "trigger-no-displacement-reset": ("for (int64_t k = 0; k < 3 * n; ++k) disp[k] = 0.0;\n            }",
                                      "for (int64_t k = 0; k < 3 * n; ++k) (void)disp[k];\n            }"),
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
    run("fs-vanishes", pins.test_force_shifted_vanishes_at_rc, 1.0, 1.0, False)
    run("fs-integral", pins.test_force_shifted_pair_energy_is_integral_of_force)
    run("fs-gradient", pins.test_force_shifted_is_minus_gradient, 4)
    run("fs-lattice-sum", pins.test_force_shifted_lattice_sum, 0.85, 2.5, 5)
    run("full-vs-half", pins.test_full_list_forces_equal_half_list, "disordered", 0)
    run("sample-rows", pins.test_sample_rows_and_virial_match_the_lists, "lj4k")
    run("nve-trigger", pins.test_nve_trigger_keeps_every_pair)
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
