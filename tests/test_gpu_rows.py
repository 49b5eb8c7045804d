"""GPU parity of the dense-rows path (sn_load_dense_rows_i8, SN_PATH_DENSE_ROWS)
against the CPU oracle, bit for bit.

Small and ragged nets run against the whole-network dense oracle; the
paper-scale net (N = 100,000 all-to-all) is checked on sampled neurons: the
oracle recomputes each sampled neuron's spikes and final state from the GPU's
own raster (every other neuron's spikes), which must reproduce the GPU's
column of that raster exactly.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2305_02510_amd import workloads as wl  # noqa: E402
from test_gpu_parity import assert_parity  # noqa: E402
from test_oracle_columns import STRONG  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_02510_amd import Network
    return Network


def rows_run(Network, net, chunks=None, path="auto", posts=None):
    g, cols = Network.from_rows_workload(net, posts=posts)
    g.set_path(path)
    for c in (chunks or [net.steps]):
        g.run(c)
    spikes = g.read_raster(0, net.steps)
    V, ref = g.read_state()
    used = g.progress[1]
    g.close()
    return spikes, V, ref, used, cols


@pytest.mark.parametrize("n,trials,steps,seed", [(1000, 1, 120, 21), (777, 3, 40, 22), (64, 1, 50, 23),
                                                 (257, 2, 33, 24), (1, 1, 10, 25)])
def test_rows_parity(gpu, oracle, n, trials, steps, seed):
    net = wl.paper_scale_dense(seed=seed, n=n, trials=trials, steps=steps, drive_p=0.06, **STRONG)
    print(f"rows parity n={n} trials={trials} steps={steps} seed={seed}", flush=True)
    res = oracle.run_dense(net, W=net.dense())
    s, V, r, used, _ = rows_run(gpu, net)
    assert used == "dense_rows"
    assert_parity(net, res, s, V, r, "dense_rows")
    if n >= 257:
        assert (res.spikes & (1 - net.ext)).sum() > 0, "recurrent spikes expected"


def test_rows_resumable(gpu, oracle):
    net = wl.paper_scale_dense(seed=26, n=500, trials=2, steps=80, drive_p=0.06, **STRONG)
    res = oracle.run_dense(net, W=net.dense())
    s, V, r, used, _ = rows_run(gpu, net, chunks=[1, 30, 49], path="dense_rows")
    assert used == "dense_rows"
    assert_parity(net, res, s, V, r, "dense_rows in pieces")


def test_rows_list_rounds(gpu, oracle):
    # every neuron driven at step 0: 12,000 spiking rows at step 1, more than
    # one round of the workgroup's spike list
    net = wl.paper_scale_dense(seed=27, n=12000, trials=1, steps=6)
    net.ext[:, 0, :] = 1
    res = oracle.run_dense(net, W=net.dense())
    assert res.spikes[0, 0].sum() == 12000
    s, V, r, _, _ = rows_run(gpu, net)
    assert_parity(net, res, s, V, r, "dense_rows, 12,000 spikes in one step")


def test_rows_paper_scale_sampled(gpu, oracle):
    # the paper's largest net at full size, in the launch configuration the
    # benchmark times; sampled neurons against the oracle, one by one
    n, steps = 100_000, 200
    net = wl.paper_scale_dense(n=n, steps=steps)
    rng = np.random.default_rng(5)
    posts = np.unique(np.concatenate([[0, 1, 63, 64, 255, 256, n - 2, n - 1],
                                      rng.choice(n, 40, replace=False)])).astype(np.int32)
    print(f"rows paper scale n={n} steps={steps} sampled={posts.size}", flush=True)
    s, V, r, used, cols = rows_run(gpu, net, posts=posts)
    assert used == "dense_rows"
    rate = s.mean()
    assert 0.002 < rate < 0.2, f"firing rate {rate}"
    res = oracle.run_columns(net, posts, cols.astype(np.float64) / 64.0, s)
    assert res.exact
    np.testing.assert_array_equal(s[:, :, posts], res.spikes)
    np.testing.assert_array_equal(V[:, posts].astype(np.float64), res.V)
    np.testing.assert_array_equal(r[:, posts].astype(np.int32), res.ref)


def test_rows_max_neurons_sampled(gpu, oracle):
    # the largest net the rows path takes (131,072 neurons: one raster row is
    # exactly the 2048 words a workgroup lists in one pass), 17 GB of weights
    n, steps = 131072, 30
    net = wl.paper_scale_dense(seed=29, n=n, steps=steps)
    posts = np.array([0, 1, 64, 65535, 65536, n - 64, n - 2, n - 1], np.int32)
    print(f"rows max neurons n={n} steps={steps}", flush=True)
    s, V, r, used, cols = rows_run(gpu, net, posts=posts)
    assert used == "dense_rows"
    res = oracle.run_columns(net, posts, cols.astype(np.float64) / 64.0, s)
    assert res.exact
    np.testing.assert_array_equal(s[:, :, posts], res.spikes)
    np.testing.assert_array_equal(V[:, posts].astype(np.float64), res.V)
    np.testing.assert_array_equal(r[:, posts].astype(np.int32), res.ref)


def test_rows_rules_of_use(gpu, oracle):
    from paper_2305_02510_amd._lib import SnError
    Network = gpu
    net = wl.paper_scale_dense(seed=28, n=300, trials=1, steps=40, drive_p=0.06, **STRONG)
    g, _ = Network.from_rows_workload(net)
    k = net.rows(0, 10)
    with pytest.raises(SnError, match="SN_EINVAL"):
        g.load_dense_rows_i8(0, k, 5)           # exponent differs from the loaded rows
    with pytest.raises(SnError, match="SN_ERANGE"):
        g.load_dense_rows_i8(295, k, 6)         # rows past N
    with pytest.raises(SnError, match="SN_ERANGE"):
        g.load_dense_rows_i8(0, k, 25)          # exponent outside [0, 24]
    for path in ("step", "persist", "dense"):
        g.set_path(path)
        with pytest.raises(SnError, match="SN_ESTATE"):
            g.run(5)
    with pytest.raises(SnError, match="SN_ESTATE"):
        g.set_stdp(4, [1 / 64] * 4, [1 / 64] * 4, -1.0, 1.0)
    with pytest.raises(SnError, match="SN_ESTATE"):
        g.read_weights()
    g.set_path("auto")
    assert g.autotune(8)[0] == "dense_rows"
    # a synapse list replaces the rows; the sparse paths work again
    W = net.dense()
    pre, post = np.nonzero(W)
    g.load_weights_delays(pre, post, W[pre, post], np.ones(pre.shape[0], np.uint8))
    g.run(net.steps)
    res = oracle.run_dense(net, W=W)
    s = g.read_raster(0, net.steps)
    V, r = g.read_state()
    assert g.progress[1] != "dense_rows"
    g.close()
    assert_parity(net, res, s, V, r, "synapse list after rows")
    big = Network(131073)
    with pytest.raises(SnError, match="SN_ERANGE"):
        big.load_dense_rows_i8(0, np.zeros((1, 131073), np.int8), 6)
    big.close()
