"""Pins of the history-driven sparse oracle (or_lif_sparse_driven): the
update of the paper's model with the source spikes of the synaptic input
read from a given raster.

- Fixed point: fed the self-driven oracle's own raster, it returns that
  raster and the final state exactly (heterogeneous nets with duplicates,
  self-loops, several trials, delays up to D).
- Post ranges: given only the synapses into a range of post-neurons, those
  neurons' columns and states equal the whole-network result, for a random
  partition into ranges (the fan-out the GPU tests use).
- Delay and drive: one synapse i -> j of delay d and a supra-threshold
  weight, with a history in which i spikes once at t0 (i itself never spikes
  in its own simulation): j spikes at t0 + d and at no other step.
Planted mistakes in a copy of the source (history ignored, source step off by
one, synapse direction swapped) each fail one of these."""
import numpy as np
import pytest

import oracle as oracle_mod
from paper_2305_02510_amd import workloads as wl


@pytest.fixture(scope="module")
def orc():
    return oracle_mod.Oracle()


def _nets():
    yield wl.random_small(901, n=40, p=0.15, max_delay=5, steps=60, trials=3, hetero=True)
    yield wl.random_small(902, n=130, p=0.05, max_delay=9, steps=80, trials=1, hetero=True)
    yield wl.large_sparse(903, n=1500, p=0.02, steps=120)


def pin_fixed_point(o):
    for net in _nets():
        ref = o.run_sparse(net)
        got = o.run_sparse_driven(net, ref.spikes)
        assert ref.exact and got.exact
        assert np.array_equal(got.spikes, ref.spikes), net.name
        assert np.array_equal(got.V, ref.V) and np.array_equal(got.ref, ref.ref), net.name


def pin_post_ranges(o):
    rng = np.random.default_rng(7)
    for net in _nets():
        ref = o.run_sparse(net)
        perm = rng.permutation(net.n)
        for part in np.array_split(perm, 3):
            posts = np.sort(part)
            got = o.run_sparse_driven(net, ref.spikes, posts=posts)
            assert np.array_equal(got.spikes[:, :, posts], ref.spikes[:, :, posts]), net.name
            assert np.array_equal(got.V[:, posts], ref.V[:, posts]), net.name
            assert np.array_equal(got.ref[:, posts], ref.ref[:, posts]), net.name


def pin_delay_and_drive(o):
    for d, t0 in [(1, 0), (3, 5), (7, 2), (16, 10)]:
        n, T = 4, 40
        th, lk, rs, rf, am = wl._params(n, 1.0, 0.25, 0.0, 2, 2.0)
        net = wl.Network(f"pair_d{d}", n, 1, 16, T, th, lk, rs, rf, am, np.array([1], np.int32),
                         np.array([2], np.int32), np.array([1.5], np.float32), np.array([d], np.uint8),
                         np.zeros((1, T, n), np.uint8))
        hist = np.zeros((1, T, n), np.uint8)
        hist[0, t0, 1] = 1
        got = o.run_sparse_driven(net, hist)
        assert np.flatnonzero(got.spikes[0, :, 2]).tolist() == [t0 + d], (d, t0)
        assert got.spikes[0, :, 1].sum() == 0  # neuron 1 has no input of its own
        assert got.spikes[0, :, [0, 3]].sum() == 0


DRIVEN_PINS = [pin_fixed_point, pin_post_ranges, pin_delay_and_drive]

DRIVEN_MUTANTS = {
    "history_ignored": ("const uint8_t* src = history ? history + (size_t)b * T * N : sb;",
                        "const uint8_t* src = sb;"),
    "source_step_off_by_one": ("int32_t src_t = t - delay[k];\n                if (src_t < 0) continue;",
                               "int32_t src_t = t - delay[k] + 1;\n                if (src_t < 0) continue;"),
    "direction_swapped": ("if (src[(size_t)src_t * N + pre[k]]) U[post[k]] += w[k];",
                          "if (src[(size_t)src_t * N + post[k]]) U[pre[k]] += w[k];"),
}


@pytest.mark.parametrize("pin", DRIVEN_PINS, ids=lambda f: f.__name__)
def test_driven_pin(orc, pin):
    pin(orc)


@pytest.mark.parametrize("name", sorted(DRIVEN_MUTANTS))
def test_driven_mutant_is_caught(name, tmp_path):
    with open(oracle_mod.SRC) as f:
        source = f.read()
    old, new = DRIVEN_MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    oracle_mod.build(str(src), str(lib))
    mutant = oracle_mod.Oracle(str(lib))
    failures = []
    for pin in DRIVEN_PINS:
        try:
            pin(mutant)
        except (AssertionError, ValueError):
            failures.append(pin.__name__)
    assert failures, f"mutant {name} passed every pin"
