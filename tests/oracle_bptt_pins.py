"""Pins of the oracle's surrogate-gradient BPTT (or_bptt).

- Finite differences: with the sigmoid-relaxed forward the oracle's gradient
  is a true gradient, so central differences of the loss (computed by the
  forward alone) must match it.
- Forward: with hard spikes, the recurrent layer is the simulation model with
  256 extra relay neurons that carry the input spikes one step ahead; the
  spike counts must equal those of the simulation oracle on that network.
- Trials: the loss is a mean over trials, so the gradient of a batch is the
  mean of the single-trial gradients.
"""
from __future__ import annotations

import numpy as np

from paper_2305_02510_amd.workloads import Network


def small_problem(seed, N=12, Nin=5, B=3, T=25, dyadic=False):
    g = np.random.default_rng(seed)
    if dyadic:
        W_rec = g.integers(-24, 40, size=(N, N)) / 64.0
        W_in = g.integers(0, 64, size=(Nin, N)) / 64.0
    else:
        W_rec = g.normal(0.05, 0.35, size=(N, N))
        W_in = g.uniform(0.2, 1.0, size=(Nin, N))
    x = (g.random((T, B, Nin)) < 0.3).astype(np.uint8)
    target = g.uniform(0.0, 0.3, size=N)
    return W_rec, W_in, x, target


def pin_bptt_finite_differences(oracle):
    for seed in range(3):
        W_rec, W_in, x, target = small_problem(100 + seed)
        res = oracle.bptt(W_rec, W_in, x, target, relaxed=True)
        g = np.random.default_rng(seed)
        eps = 1e-6
        for which, W, dW in (("rec", W_rec, res.dW_rec), ("in", W_in, res.dW_in)):
            for _ in range(6):
                i, j = g.integers(0, W.shape[0]), g.integers(0, W.shape[1])
                Wp, Wm = W.copy(), W.copy()
                Wp[i, j] += eps
                Wm[i, j] -= eps
                if which == "rec":
                    lp = oracle.bptt(Wp, W_in, x, target, relaxed=True).loss
                    lm = oracle.bptt(Wm, W_in, x, target, relaxed=True).loss
                else:
                    lp = oracle.bptt(W_rec, Wp, x, target, relaxed=True).loss
                    lm = oracle.bptt(W_rec, Wm, x, target, relaxed=True).loss
                fd = (lp - lm) / (2 * eps)
                scale = max(abs(fd), 1e-3 * np.abs(dW).max(), 1e-12)
                assert abs(fd - dW[i, j]) <= 1e-5 * scale, f"W_{which}[{i},{j}]: fd {fd} vs {dW[i, j]}"


def embedded_network(W_rec, W_in, x, theta=1.0, leak=0.0625):
    """The recurrent layer as a delay-1 simulation net: neurons 0..Nin-1 relay
    the inputs (spiked externally one step early, amplitude above threshold,
    no leak influence at rest), neurons Nin.. are the layer."""
    T, B, Nin = x.shape
    N = W_rec.shape[0]
    M = Nin + N
    W = np.zeros((M, M))
    W[:Nin, Nin:] = W_in
    W[Nin:, Nin:] = W_rec
    ext = np.zeros((B, T + 1, M), np.uint8)
    ext[:, :T, :Nin] = x.transpose(1, 0, 2)
    f32 = lambda v: np.full(M, v, np.float32)
    pre, post = np.nonzero(W)
    return Network("bptt_embedded", M, B, 1, T + 1, f32(theta), f32(leak), f32(0.0), np.zeros(M, np.uint8),
                   f32(2.0), pre.astype(np.int32), post.astype(np.int32), W[pre, post].astype(np.float32),
                   np.ones(pre.shape[0], np.uint8), ext, dense_weight=W.astype(np.float32))


def pin_bptt_forward_is_simulation(oracle):
    for seed in range(3):
        W_rec, W_in, x, target = small_problem(200 + seed, dyadic=True)
        res = oracle.bptt(W_rec, W_in, x, target, relaxed=False)
        sim = oracle.run_dense(embedded_network(W_rec, W_in, x))
        Nin = W_in.shape[0]
        counts = sim.spikes[:, 1:, Nin:].sum(axis=1)
        assert np.array_equal(res.counts, counts), f"seed {seed}: spike counts differ"
        assert res.counts.sum() > 0


def pin_bptt_trial_mean(oracle):
    W_rec, W_in, x, target = small_problem(300, B=4)
    full = oracle.bptt(W_rec, W_in, x, target, relaxed=False)
    parts = [oracle.bptt(W_rec, W_in, x[:, b:b + 1], target, relaxed=False) for b in range(4)]
    assert np.allclose(full.dW_rec, np.mean([p.dW_rec for p in parts], 0), rtol=1e-12, atol=1e-15)
    assert np.allclose(full.dW_in, np.mean([p.dW_in for p in parts], 0), rtol=1e-12, atol=1e-15)
    assert abs(full.loss - np.mean([p.loss for p in parts])) < 1e-14


ALL_BPTT_PINS = [pin_bptt_finite_differences, pin_bptt_forward_is_simulation, pin_bptt_trial_mean]
