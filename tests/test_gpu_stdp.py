"""Plasticity on the GPU (sn_set_stdp, per-step path) against the oracle's
rule: rasters, final state and final weights bit for bit."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from paper_2305_02510_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

LTP = [16 / 64, 8 / 64, 4 / 64, 2 / 64, 1 / 64, 1 / 64, 1 / 64, 1 / 64]
LTD = [12 / 64, 6 / 64, 3 / 64, 2 / 64, 1 / 64, 1 / 64, 1 / 64, 1 / 64]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_02510_amd import Network
    return Network


def run_stdp(Network, net, window, w_min, w_max, chunks):
    g = Network.from_workload(net)
    g.set_stdp(window, LTP, LTD, w_min, w_max)
    for c in chunks:
        g.run(c)
    spikes = g.read_raster(0, net.steps)[0]
    V, ref = g.read_state()
    w = g.read_weights()
    path = g.progress[1]
    g.close()
    return spikes, V[0], ref[0], w, path


def check(net, res, spikes, V, ref, w, what):
    assert res.exact, f"{what}: input violates the exactness premise"
    if not np.array_equal(spikes, res.spikes):
        t, j = np.argwhere(spikes != res.spikes)[0]
        raise AssertionError(f"{what}: raster differs first at step {t} neuron {j}")
    assert np.array_equal(V.astype(np.float64), res.V), f"{what}: V differs"
    assert np.array_equal(ref.astype(np.int32), res.ref), f"{what}: refractory counters differ"
    bad = np.flatnonzero(w.astype(np.float64) != res.weight)
    assert bad.size == 0, f"{what}: {bad.size} weights differ, first synapse {bad[:1]}"


@pytest.mark.parametrize("seed,n,window,chunks", [(1, 60, 5, [20, 100]), (2, 250, 8, [40, 80]),
                                                   (3, 130, 1, [120]), (4, 300, 3, [7, 33, 80])])
def test_stdp_small_nets(gpu, oracle, seed, n, window, chunks):
    net = wl.random_small(600 + seed, n=n, p=0.08, max_delay=4, steps=sum(chunks), drive_p=0.15)
    res = oracle.stdp(net, window, LTP, LTD, -1.0, 1.5)
    assert (res.weight != net.weight).any(), "the rule changed no weight: a weak test"
    out = run_stdp(gpu, net, window, -1.0, 1.5, chunks)
    assert out[4] == "step"
    check(net, res, *out[:4], f"seed={seed} n={n} window={window}")


def test_stdp_long_delays(gpu, oracle):
    """Delays up to 64 with window 8: records with d + W > 64 look past the
    64-step history words and take the raster rows instead."""
    net = wl.random_small(620, n=120, p=0.15, max_delay=64, steps=200, drive_p=0.15)
    assert (net.delay.astype(int) + 8 > 64).any()
    res = oracle.stdp(net, 8, LTP, LTD, -1.0, 1.5)
    assert (res.weight != net.weight).any()
    out = run_stdp(gpu, net, 8, -1.0, 1.5, [70, 130])
    check(net, res, *out[:4], "long delays")


def test_stdp_larger_net(gpu, oracle):
    """N = 3000, p = 0.02 (about 180k synapses), delays 1..16, 150 steps."""
    net = wl.large_sparse(21, n=3000, p=0.02, steps=150)
    res = oracle.stdp(net, 8, LTP, LTD, -0.5, 1.0)
    out = run_stdp(gpu, net, 8, -0.5, 1.0, [50, 100])
    check(net, res, *out[:4], "large")


def test_stdp_rules_of_use(gpu, oracle):
    from paper_2305_02510_amd._lib import SnError
    net = wl.random_small(610, n=80, p=0.1, max_delay=3, steps=40)
    g = gpu.from_workload(net)
    g.set_stdp(4, LTP, LTD, -1.0, 1.5)
    g.set_path("persist")
    with pytest.raises(SnError):
        g.run(10)                       # plasticity runs on the per-step path only
    with pytest.raises(SnError):
        g.autotune(8)                   # timing would change the weights
    g.set_path("auto")
    g.run(40)
    g.stdp_off()
    g.set_path("push")
    with pytest.raises(SnError):
        g.run(5)                        # event-driven records hold the old weights
    g.close()
    two = wl.random_small(611, n=40, p=0.1, max_delay=3, steps=10, trials=2)
    g = gpu.from_workload(two)
    with pytest.raises(SnError):
        g.set_stdp(4, LTP, LTD, -1.0, 1.5)  # one trial only
    g.close()
    # weights read back without plasticity are the loaded ones
    g = gpu.from_workload(net)
    assert np.array_equal(g.read_weights(), net.weight.astype(np.float32))
    g.close()


@pytest.mark.parametrize("n,p,D", [(3000, 0.02, 16), (40_000, 0.0005, 16)])
def test_learned_weights_on_every_path(gpu, oracle, n, p, D):
    """After plasticity has changed the weights and is turned off, the paths
    that read 4-byte copies of the records (persistent kernel: compact
    records at N = 3000; wide per-step kernel: lane records at N = 40,000)
    run with the learned weights: they continue the run exactly as the
    per-step path that learned them (8-byte records) does."""
    net = wl.large_sparse(620 + n % 97, n=n, p=p, steps=100, max_delay=D)
    other = "persist" if n < 10_000 else "step"
    ref = "step" if other == "persist" else "persist"
    runs = {}
    for second in (ref, other):
        g = gpu.from_workload(net)
        g.set_stdp(4, LTP, LTD, -1.0, 1.5)
        g.set_path("step")
        g.run(40)
        learned = g.read_weights()
        g.stdp_off()
        g.set_path(second)
        g.run(60)
        assert g.progress[1] == second
        runs[second] = (g.read_raster(0, 100), *g.read_state(), learned)
        g.close()
    assert not np.array_equal(runs[ref][3], net.weight.astype(np.float32)), "the rule changed no weight"
    for a, b in zip(runs[ref], runs[other]):
        assert np.array_equal(a, b)


def test_batch_refuses_plasticity(gpu, oracle):
    """A batch does not apply the rule, so it refuses a net with plasticity
    on, both when planned and when the rule is turned on afterwards."""
    from paper_2305_02510_amd import Batch
    from paper_2305_02510_amd._lib import SnError
    a = gpu.from_workload(wl.random_small(612, n=60, p=0.1, max_delay=3, steps=20))
    b = gpu.from_workload(wl.random_small(613, n=90, p=0.1, max_delay=2, steps=20))
    b.set_stdp(4, LTP, LTD, -1.0, 1.5)
    with pytest.raises(SnError, match="SN_ESTATE"):
        Batch([a, b])
    b.stdp_off()
    batch = Batch([a, b])
    batch.run(5)
    b.set_stdp(4, LTP, LTD, -1.0, 1.5)
    with pytest.raises(SnError, match="SN_ESTATE"):
        batch.run(5)
    batch.close()
    a.close()
    b.close()
