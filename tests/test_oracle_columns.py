"""Pins of the oracle's column-wise dense update (or_lif_columns), which
checks large dense nets neuron by neuron against the network's own raster.

It is pinned to the whole-network dense oracle (itself pinned by the closed
forms and brute force of oracle_pins.py): fed the raster that oracle produced,
every neuron's spikes and final state must come out unchanged; and to a closed
form for one delivered spike (index order and timing).  Planted mistakes in a
copy of its C source must each fail a pin.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle as oracle_mod  # noqa: E402
from paper_2305_02510_amd import workloads as wl  # noqa: E402

# byte tables strong enough for recurrent activity in small nets
STRONG = dict(exc={0: 32, 2: 64, 4: 96, 8: 64}, inh={-12: 128, -20: 128})


def small_rows_net(n=300, trials=2, steps=60, seed=11):
    return wl.paper_scale_dense(seed=seed, n=n, trials=trials, steps=steps, drive_p=0.06, **STRONG)


def pin_columns_match_dense(orc):
    net = small_rows_net()
    W = net.dense()
    full = orc.run_dense(net, W=W)
    assert full.exact
    assert (full.spikes & (1 - net.ext)).sum() > 200, "recurrent activity expected"
    posts = np.array([0, 1, 63, 64, 150, 298, 299], np.int32)
    col = orc.run_columns(net, posts, W[:, posts].T, full.spikes)
    assert col.exact
    np.testing.assert_array_equal(col.spikes, full.spikes[:, :, posts])
    np.testing.assert_array_equal(col.V, full.V[:, posts])
    np.testing.assert_array_equal(col.ref, full.ref[:, posts])


def pin_columns_single_arrival(orc):
    # one spike of pre-neuron i at step 0 in the given history, no external
    # input: at rest (V = r = 0) neuron j holds exactly W[i][j] after step 1
    net = small_rows_net(n=40, trials=1, steps=2)
    net.ext[:] = 0
    W = net.dense()
    i = 7
    hist = np.zeros((1, 2, net.n), np.uint8)
    hist[0, 0, i] = 1
    posts = np.arange(net.n, dtype=np.int32)
    col = orc.run_columns(net, posts, W.T, hist)
    expect = np.where(W[i] > 1.0, 0.0, W[i])  # above threshold: spike and reset to 0
    np.testing.assert_array_equal(col.V[0], expect)
    np.testing.assert_array_equal(col.spikes[0, 1], (W[i] > 1.0).astype(np.uint8))
    assert (col.spikes[0, 0] == 0).all()
    one = orc.run_columns(net, posts, W.T, hist, steps=1)
    np.testing.assert_array_equal(one.V[0], np.zeros(net.n))


COLUMN_PINS = [pin_columns_match_dense, pin_columns_single_arrival]

COLUMN_MUTANTS = {
    "same_step_history": ("const size_t bt = (size_t)b * T + (t - 1);",
                          "const size_t bt = (size_t)b * T + t;"),
    "external_of_slot": ("if (xb[(size_t)t * N + j]) U += amplitude[j];",
                         "if (xb[(size_t)t * N + k]) U += amplitude[j];"),
    "no_leak": ("double U = apply_leak(V, reset[j], leak[j]);", "double U = V;"),
    "state_not_reset_per_trial": ("            double V = reset[j];\n            int32_t ref = 0;",
                                  "            static double V = 0.0;\n            static int32_t ref = 0;"),
}


@pytest.fixture(scope="module")
def orc():
    return oracle_mod.Oracle()


@pytest.mark.parametrize("pin", COLUMN_PINS, ids=lambda p: p.__name__)
def test_column_pin(orc, pin):
    pin(orc)


@pytest.mark.parametrize("name", sorted(COLUMN_MUTANTS))
def test_column_mutant_is_caught(name, tmp_path):
    with open(oracle_mod.SRC) as f:
        source = f.read()
    old, new = COLUMN_MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    oracle_mod.build(str(src), str(lib))
    mutant = oracle_mod.Oracle(str(lib))
    failures = []
    for pin in COLUMN_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, f"mutant {name} passed every pin"
