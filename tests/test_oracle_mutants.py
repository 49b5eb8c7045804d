"""The pins must be strong enough to catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (a flipped
comparison, a wrong sign, an off-by-one delay, a transposed synapse, ...),
compiles it into a temporary directory and runs every pin against it; at least
one pin must fail.  The real oracle is never modified.
"""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle as oracle_mod  # noqa: E402
from oracle_pins import ALL_PINS  # noqa: E402

MUTANTS = {
    "threshold_ge": ("int candidate = u > theta;", "int candidate = u >= theta;"),
    "leak_sign_above": ("double u = v - lambda;", "double u = v + lambda;"),
    "leak_sign_below": ("double u = v + lambda;", "double u = v - lambda;"),
    "leak_no_clamp_above": ("return u < r ? r : u;", "return u;"),
    "leak_no_clamp_below": ("return u > r ? r : u;", "return u;"),
    "leak_towards_zero": ("apply_leak(V[j], reset[j], leak[j])", "apply_leak(V[j], 0.0, leak[j])"),
    "delay_plus_one": ("int32_t src_t = t - delay[k];", "int32_t src_t = t - delay[k] - 1;"),
    "delay_minus_one": ("int32_t src_t = t - delay[k];", "int32_t src_t = t - delay[k] + 1;"),
    "delay_ignored": ("int32_t src_t = t - delay[k];", "int32_t src_t = t - 1;"),
    "transposed": ("if (src[(size_t)src_t * N + pre[k]]) U[post[k]] += w[k];",
                   "if (src[(size_t)src_t * N + post[k]]) U[pre[k]] += w[k];"),
    "unit_weight": ("U[post[k]] += w[k];", "U[post[k]] += 1.0;"),
    "external_dropped": ("U[j] += amplitude[j];", "U[j] += 0.0;"),
    "external_late": ("if (xb[(size_t)t * N + j]) U[j] += amplitude[j];",
                      "if (t > 0 && xb[(size_t)(t - 1) * N + j]) U[j] += amplitude[j];"),
    "refractory_stuck": ("*ref = *ref - 1;", "*ref = *ref;"),
    "refractory_long": ("*ref = R;", "*ref = R + 1;"),
    "refractory_short": ("if (*ref > 0) {", "if (*ref > 1) {"),
    "refractory_holds_reset": ("        spike = 0;\n        *ref = *ref - 1;",
                               "        spike = 0;\n        *ref = *ref - 1;\n        u = r;"),
    "reset_to_zero": ("        *v = r;\n        *ref = R;", "        *v = 0.0;\n        *ref = R;"),
    "no_reset": ("        *v = r;\n        *ref = R;", "        *v = u;\n        *ref = R;"),
    "threshold_of_neuron0": ("fire_and_reset(U[j], theta[j],", "fire_and_reset(U[j], theta[0],"),
    "trials_share_state": ("double* V = V_out + (size_t)b * N;", "double* V = V_out;"),
    "leak_dropped": ("U[j] = apply_leak(V[j], reset[j], leak[j]);", "U[j] = V[j];"),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle_mod.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert old in source, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    oracle_mod.build(str(src), str(lib))
    mutant = oracle_mod.Oracle(str(lib))
    failures = []
    for pin in ALL_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, f"mutant {name} passed every pin"
