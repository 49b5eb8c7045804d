"""The oracle's surrogate-gradient BPTT against finite differences, the
simulation oracle and trial additivity; planted mistakes must be caught."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle as oracle_mod  # noqa: E402
from oracle_bptt_pins import ALL_BPTT_PINS  # noqa: E402


@pytest.mark.parametrize("pin", ALL_BPTT_PINS, ids=[p.__name__ for p in ALL_BPTT_PINS])
def test_bptt_pin(oracle, pin):
    pin(oracle)


BPTT_MUTANTS = {
    "surrogate_sign": ("return 1.0 / (d * d);", "return -1.0 / (d * d);"),
    "surrogate_scaled": ("return 1.0 / (d * d);", "return 0.5 * k / (d * d);"),
    "surrogate_not_squared": ("return 1.0 / (d * d);", "return 1.0 / d;"),
    "no_reset_term": ("gcur[i] = a * sg + gv * ((1.0 - st[i]) + (r - Ut[i]) * sg);",
                      "gcur[i] = a * sg + gv * (1.0 - st[i]);"),
    "leak_always_passes": ("double gv = fabs(Vt[i] - r) > lambda ? gnext[i] : 0.0;", "double gv = gnext[i];"),
    "recurrence_transposed": ("for (int32_t j = 0; j < N; ++j) a += gnext[j] * W_rec[(size_t)i * N + j];",
                              "for (int32_t j = 0; j < N; ++j) a += gnext[j] * W_rec[(size_t)j * N + i];"),
    "loss_scale": ("double a = 2.0 * (counts[(size_t)b * N + i] / T - target[i]) / ((double)B * N * T);",
                   "double a = 2.0 * (counts[(size_t)b * N + i] / T - target[i]) / ((double)B * N);"),
    "input_gradient_halved": ("for (int32_t j = 0; j < N; ++j) dW_in[(size_t)i * N + j] += gcur[j];",
                              "for (int32_t j = 0; j < N; ++j) dW_in[(size_t)i * N + j] += 0.5 * gcur[j];"),
    "recurrent_gradient_same_step": ("const double* sp = s + ((size_t)(t - 1) * B + b) * N;\n                for (int32_t i = 0; i < N; ++i) {\n                    if (sp[i] == 0.0) continue;\n                    for (int32_t j = 0; j < N; ++j) dW_rec",
                                     "const double* sp = s + ((size_t)(t) * B + b) * N;\n                for (int32_t i = 0; i < N; ++i) {\n                    if (sp[i] == 0.0) continue;\n                    for (int32_t j = 0; j < N; ++j) dW_rec"),
    "relaxed_scale": ("return 0.5 + x / (1.0 + k * fabs(x));", "return 0.5 + 0.5 * k * x / (1.0 + k * fabs(x));"),
    "hard_ge": ("(Ut[j] > theta ? 1.0 : 0.0)", "(Ut[j] >= theta ? 1.0 : 0.0)"),
}


@pytest.mark.parametrize("name", sorted(BPTT_MUTANTS))
def test_bptt_mutant_is_caught(name, tmp_path):
    src_text = open(oracle_mod.SRC).read()
    old, new = BPTT_MUTANTS[name]
    assert old in src_text, name
    src = tmp_path / "mutant.c"
    src.write_text(src_text.replace(old, new))
    lib = tmp_path / "libmutant.so"
    oracle_mod.build(str(src), str(lib))
    mutant = oracle_mod.Oracle(str(lib))
    failures = []
    for pin in ALL_BPTT_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, f"mutant {name} passed every BPTT pin"
