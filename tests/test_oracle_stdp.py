"""The oracle's plasticity rule against closed forms and a second
transcription (oracle_stdp_pins.py), and mutants of it that the pins catch."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_stdp_pins import ALL_STDP_PINS  # noqa: E402

import oracle  # noqa: E402

# (original text, replacement) in or_lif_stdp
STDP_MUTANTS = {
    "ltd_sign": ("change -= ltd[lag - 1]; break;", "change += ltd[lag - 1]; break;"),
    "ltp_ignores_delay": ("int32_t tau = t - lag - d;", "int32_t tau = t - lag;"),
    "ltp_window_inclusive": ("for (int32_t lag = 0; lag < W; ++lag) {   /* arrival", "for (int32_t lag = 0; lag <= W; ++lag) {   /* arrival"),
    "ltd_same_step": ("for (int32_t lag = 1; lag <= W; ++lag) {  /* post spike", "for (int32_t lag = 0; lag <= W; ++lag) {  /* post spike"),
    "ltd_index": ("change -= ltd[lag - 1]; break;", "change -= ltd[lag < W ? lag : W - 1]; break;"),
    "no_clip": ("w[k] = x < w_min ? w_min : (x > w_max ? w_max : x);", "w[k] = x;"),
    "all_pairs": ("if (spikes[(size_t)tau * N + i]) { change += ltp[lag]; break; }", "if (spikes[(size_t)tau * N + i]) { change += ltp[lag]; }"),
}


def test_stdp_pins(oracle):
    for pin in ALL_STDP_PINS:
        pin(oracle)


@pytest.fixture(scope="module")
def source():
    return open(oracle.SRC).read()


@pytest.mark.parametrize("name", sorted(STDP_MUTANTS))
def test_stdp_mutant_is_caught(name, source, tmp_path):
    old, new = STDP_MUTANTS[name]
    assert source.count(old) == 1, name
    src = tmp_path / "m.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "m.so"
    oracle.build(str(src), str(lib))
    mutant = oracle.Oracle(str(lib))
    caught = False
    for pin in ALL_STDP_PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name} passes every pin"
