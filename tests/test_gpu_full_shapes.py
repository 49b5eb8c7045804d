"""GPU parity at the full sizes the benchmark times, in its launch
configuration, against the CPU oracle fanned out over the host's cores (one
single-threaded oracle run per trial, net or column chunk).

- dense trials: N = 4096, 64 trials, T = 1000, every trial;
- uneven batch: all 512 nets, T = 500, in one batched launch;
- surrogate-gradient BPTT: N = 2048, 256 inputs, 128 trials, T = 200,
  checkpoints every 50 steps (two 64-trial tiles and the large-batch K split);
- dense rows above 2^31 bytes of weights (N = 50,000): every neuron's column
  recomputed by the column oracle from the GPU raster.  Each column's spikes
  at step t depend only on the raster before t, so when every column matches,
  induction over t makes the raster the oracle's own: whole-network parity.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2305_02510_amd import workloads as wl  # noqa: E402
from test_gpu_parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_02510_amd import Network
    return Network


def test_dense_trials_every_trial(gpu, oracle):
    import oracle as om
    net = wl.dense_trials(3)
    print(f"dense trials full: N={net.n} B={net.trials} T={net.steps}", flush=True)
    g = gpu.from_workload(net)
    g.autotune(128)  # as the benchmark: the autotuner's path
    g.run(net.steps)
    used = g.progress[1]
    spikes = g.read_raster(0, net.steps)
    V, ref = g.read_state()
    g.close()
    W = np.ascontiguousarray(net.dense_weight, np.float64)
    parts = om.fan_out(lambda b: oracle.run_dense(net, trials=[b], W=W), range(net.trials))
    for b, res in enumerate(parts):
        assert res.exact
        if not np.array_equal(spikes[b], res.spikes[0]):
            t, j = np.argwhere(spikes[b] != res.spikes[0])[0]
            raise AssertionError(f"{used}: trial {b} differs first at step {t} neuron {j}")
        assert np.array_equal(V[b].astype(np.float64), res.V[0]), f"{used}: V of trial {b}"
        assert np.array_equal(ref[b].astype(np.int32), res.ref[0]), f"{used}: counters of trial {b}"
    assert 0.001 < spikes.mean() < 0.2


def test_uneven_batch_every_net(gpu, oracle):
    import oracle as om
    from paper_2305_02510_amd import Batch
    nets = wl.uneven_batch(4)
    T = nets[0].steps
    print(f"uneven batch full: {len(nets)} nets, T={T}, nnz={sum(n.nnz for n in nets)}", flush=True)
    gs = [gpu.from_workload(net) for net in nets]
    batch = Batch(gs)
    batch.run(T)
    batch.synchronize()
    got = []
    for g in gs:
        assert g.progress == (T, "batch")
        got.append((g.read_raster(0, T), *g.read_state()))
    batch.close()
    for g in gs:
        g.close()
    order = sorted(range(len(nets)), key=lambda i: -nets[i].nnz)  # longest first
    results = dict(zip(order, om.fan_out(lambda i: oracle.run_sparse(nets[i]), order)))
    for i, net in enumerate(nets):
        assert_parity(net, results[i], *got[i], f"batch net {i}")


def test_bptt_full_batch(oracle):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle as om
    from test_gpu_bptt import gpu_grad, rel_err
    prob = wl.bptt_problem(5)
    T, B, _ = prob.x.shape
    print(f"bptt full: N={prob.W_rec.shape[0]} B={B} T={T} K={prob.checkpoint}", flush=True)
    counts, loss, gWr, gWi = gpu_grad(torch, prob)
    # the loss is a mean over trials and neurons, so the batch gradient is the
    # trial-count-weighted mean of the gradients of trial subsets
    chunks = [list(range(i, min(B, i + 8))) for i in range(0, B, 8)]
    parts = om.fan_out(lambda tr: oracle.bptt(prob.W_rec, prob.W_in, prob.x[:, tr], prob.target, prob.theta,
                                              prob.leak, prob.reset, prob.slope), chunks)
    dWr = sum(len(tr) / B * p.dW_rec for tr, p in zip(chunks, parts))
    dWi = sum(len(tr) / B * p.dW_in for tr, p in zip(chunks, parts))
    ref_loss = sum(len(tr) / B * p.loss for tr, p in zip(chunks, parts))
    ref_counts = np.concatenate([p.counts for p in parts])
    assert np.array_equal(counts, ref_counts), "hard-spike forward must be exact (dyadic weights)"
    assert abs(loss - ref_loss) <= 1e-6 * ref_loss
    assert rel_err(gWr, dWr) <= 1e-4, rel_err(gWr, dWr)
    assert rel_err(gWi, dWi) <= 1e-4, rel_err(gWi, dWi)


def test_rows_beyond_2gib_every_column(gpu, oracle):
    import oracle as om
    n, steps, chunk = 50_000, 200, 512
    net = wl.paper_scale_dense(seed=30, n=n, steps=steps)
    print(f"dense rows, every column: N={n} T={steps} ({n * ((n + 63) // 64 * 64)} bytes of rows)", flush=True)
    g, _ = gpu.from_rows_workload(net, workers=om.host_workers())
    g.run(steps)
    assert g.progress[1] == "dense_rows"
    s = g.read_raster(0, steps)
    V, ref = g.read_state()
    g.close()
    assert 0.002 < s.mean() < 0.2, s.mean()
    k = np.empty((n, n), np.int8)

    def fill(bi):
        kb = net.block(bi)
        k[bi * net.block_rows:bi * net.block_rows + kb.shape[0]] = kb

    om.fan_out(fill, range(net.n_blocks))
    scale = 2.0 ** -net.e

    def columns(c0):
        c1 = min(n, c0 + chunk)
        res = oracle.run_columns(net, np.arange(c0, c1, dtype=np.int32), k[:, c0:c1].T.astype(np.float64) * scale, s)
        ok = (res.exact and np.array_equal(s[:, :, c0:c1], res.spikes)
              and np.array_equal(V[:, c0:c1].astype(np.float64), res.V)
              and np.array_equal(ref[:, c0:c1].astype(np.int32), res.ref))
        return c0, ok

    bad = [c0 for c0, ok in om.fan_out(columns, range(0, n, chunk)) if not ok]
    assert not bad, f"columns starting at {bad[:8]} differ from the oracle"


@pytest.mark.parametrize("p", [0.001, 0.01])
def test_sparse_xl_every_post_range(gpu, oracle, p):
    """N = 100,000 sparse nets (1e7 and 1e8 synapses, records far beyond
    LDS), on the path the autotuner picks; every post range recomputed by the
    history-driven oracle from the GPU raster (all ranges = whole-network
    parity, by induction over t)."""
    import oracle as om
    steps = 200
    net = wl.large_sparse_xl(p=p, steps=steps)
    print(f"sparse xl: N={net.n} p={p} nnz={net.nnz} T={steps}", flush=True)
    g = gpu.from_workload(net)
    path, slices = g.autotune(64)
    g.run(steps)
    assert g.progress[1] == path
    s = g.read_raster(0, steps)
    V, ref = g.read_state()
    g.close()
    print(f"sparse xl: path {path}/{slices}, rate {s.mean():.4f}", flush=True)
    assert 0.05 < s.mean() < 0.5

    def check(rng):
        j0, j1, idx = rng
        res = oracle.run_sparse_driven(net, s, syn_index=idx)
        return (res.exact and np.array_equal(s[:, :, j0:j1], res.spikes[:, :, j0:j1])
                and np.array_equal(V[:, j0:j1].astype(np.float64), res.V[:, j0:j1])
                and np.array_equal(ref[:, j0:j1].astype(np.int32), res.ref[:, j0:j1])), j0
    ranges = om.post_ranges(net, 4 * om.host_workers())
    bad = [j0 for ok, j0 in om.fan_out(check, ranges) if not ok]
    assert not bad, f"post ranges starting at {bad[:8]} differ from the oracle ({path})"
