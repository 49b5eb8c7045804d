"""Seeded workload generators: determinism, dyadic values, graph statistics."""
import numpy as np

from paper_2305_02510_amd import workloads as wl


def _same(a, b):
    for f in ("threshold", "leak", "reset", "refractory", "amplitude", "pre", "post", "weight", "delay", "ext"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_deterministic():
    _same(wl.single_lif(1), wl.single_lif(1))
    _same(wl.large_sparse(5, n=1500, steps=20), wl.large_sparse(5, n=1500, steps=20))
    a, b = wl.single_lif(1), wl.single_lif(2)
    assert not np.array_equal(a.ext, b.ext)


def _dyadic(x):
    x = np.asarray(x, np.float64)
    return np.all(np.isfinite(x)) and np.all(x * 64 == np.floor(x * 64))


def test_single_lif_shape():
    net = wl.single_lif(1)
    net.validate()
    assert net.n == 110 and net.steps == 100 and net.max_delay == 3
    assert net.post.max() < 100, "input neurons 100..109 receive no synapses"
    assert not np.any(net.pre == net.post)
    assert _dyadic(net.weight) and net.weight.min() >= -1 and net.weight.max() <= 2
    assert set(np.unique(net.delay)) <= {1, 2, 3}
    assert not net.ext[:, :, :100].any() and net.ext[:, :, 100:].any()
    assert abs(net.nnz - 0.1 * (110 * 100 - 100)) < 5 * np.sqrt(0.1 * 0.9 * 10900)


def test_er_statistics():
    n, p = 3000, 0.01
    net = wl.large_sparse(7, n=n, p=p, steps=10)
    net.validate()
    m = n * (n - 1)
    assert abs(net.nnz - m * p) < 5 * np.sqrt(m * p * (1 - p))
    assert not np.any(net.pre == net.post)
    key = net.pre.astype(np.int64) * n + net.post
    assert np.unique(key).size == key.size, "no duplicate edges"
    assert _dyadic(net.weight) and net.weight.min() >= -0.5 and net.weight.max() <= 1.0
    assert net.delay.min() >= 1 and net.delay.max() <= 16
    driven = np.nonzero(net.ext[0].any(0))[0]
    assert driven.size <= 150


def test_er_dense_and_edge_cases():
    pre, post = wl.erdos_renyi_edges(20, 1.0, wl.rng_for(1, "edge"))
    assert pre.size == 20 * 19
    pre, post = wl.erdos_renyi_edges(20, 0.0, wl.rng_for(1, "edge"))
    assert pre.size == 0


def test_dense_weights():
    g1, g2 = wl.rng_for(3, "w"), wl.rng_for(3, "sel")
    W = wl.balanced_dense_weights(512, g1, g2)
    assert _dyadic(W) and np.abs(W).max() <= 0.25
    assert np.all(np.diag(W) == 0)
    rows_neg = (W <= 0).all(1)
    rows_pos = (W >= 0).all(1)
    assert np.all(rows_neg | rows_pos), "Dale's law: every row has one sign"
    assert abs(rows_neg.sum() - 0.2 * 512) <= 2 + (W.sum(1) == 0).sum()
    # bf16 represents every weight exactly (|k| <= 16)
    assert np.all(np.abs(W * 64) <= 16)


def test_uneven_batch_small():
    nets = wl.uneven_batch(4, count=6, steps=5, n_range=(50, 400))
    for net in nets:
        net.validate()
        assert 50 <= net.n <= 400
        assert _dyadic(net.threshold) and _dyadic(net.leak) and _dyadic(net.weight)


def test_rows_network_blocks():
    net = wl.paper_scale_dense(n=700, steps=5)
    k = net.rows(0, 700)
    assert k.dtype == np.int8 and k.shape == (700, 700)
    assert (np.diag(k) == 0).all()
    # any row range equals the same rows of the whole; blocks stand alone
    np.testing.assert_array_equal(net.rows(250, 530), k[250:530])
    np.testing.assert_array_equal(net.block(2), k[512:700])
    np.testing.assert_array_equal(wl.paper_scale_dense(n=700, steps=5).rows(0, 700), k)
    # row types and table values
    assert abs(net.inhibitory.mean() - 0.2) < 0.01
    assert (k[net.inhibitory] <= 0).all() and (k[~net.inhibitory] >= 0).all()
    assert set(np.unique(k[~net.inhibitory]).tolist()) <= {0, 1}
    off = ~np.eye(700, dtype=bool)
    exc_rows = off[~net.inhibitory]
    assert abs((k[~net.inhibitory] == 1).sum() / exc_rows.sum() - 0.25) < 0.01
    assert (k[net.inhibitory][off[net.inhibitory]] == -1).all()
    np.testing.assert_array_equal(net.dense(), k.astype(np.float32) / 64)
    assert abs(wl.paper_scale_dense(n=700, steps=60).ext.mean() - 0.02) < 0.003
