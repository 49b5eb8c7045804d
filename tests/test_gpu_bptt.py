"""Surrogate-gradient BPTT on the GPU against the FP64 oracle (same surrogate
definition) and against finite differences of the relaxed forward."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2305_02510_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_grad(torch, prob, trials=None, relaxed=False, checkpoint=None):
    from paper_2305_02510_amd.bptt import spike_counts
    x = prob.x if trials is None else prob.x[:, trials]
    Wr = torch.tensor(prob.W_rec, device="cuda", requires_grad=True)
    Wi = torch.tensor(prob.W_in, device="cuda", requires_grad=True)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tgt = torch.tensor(prob.target, device="cuda")
    T = x.shape[0]
    counts = spike_counts(Wr, Wi, xt, prob.theta, prob.leak, prob.reset, prob.slope,
                          checkpoint or prob.checkpoint, relaxed)
    loss = ((counts / T - tgt) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    return (counts.detach().cpu().numpy(), float(loss), Wr.grad.cpu().numpy().astype(np.float64),
            Wi.grad.cpu().numpy().astype(np.float64))


def rel_err(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,nin,trials,steps,ckpt", [(64, 16, 8, 30, 7), (96, 40, 33, 41, 50), (256, 64, 5, 80, 13)])
def test_bptt_small_vs_oracle(torch_gpu, oracle, n, nin, trials, steps, ckpt):
    prob = wl.bptt_problem(40 + n, n=n, n_in=nin, trials=trials, steps=steps, checkpoint=ckpt)
    counts, loss, gWr, gWi = gpu_grad(torch_gpu, prob)
    ref = oracle.bptt(prob.W_rec, prob.W_in, prob.x, prob.target, prob.theta, prob.leak, prob.reset, prob.slope)
    assert np.array_equal(counts, ref.counts), "hard-spike forward must be exact (dyadic weights)"
    assert abs(loss - ref.loss) <= 1e-6 * max(ref.loss, 1e-12)
    assert rel_err(gWr, ref.dW_rec) <= 1e-4, rel_err(gWr, ref.dW_rec)
    assert rel_err(gWi, ref.dW_in) <= 1e-4, rel_err(gWi, ref.dW_in)


def test_bptt_relaxed_vs_finite_differences(torch_gpu, oracle):
    """Relaxed forward, non-dyadic weights: the GPU gradient against central
    differences of the FP64 relaxed loss."""
    prob = wl.bptt_problem(77, n=64, n_in=16, trials=4, steps=25, checkpoint=6)
    g = np.random.default_rng(3)
    prob.W_rec = (prob.W_rec + g.normal(0, 0.01, prob.W_rec.shape)).astype(np.float32)
    prob.W_in = (prob.W_in + g.normal(0, 0.01, prob.W_in.shape)).astype(np.float32)
    _, _, gWr, gWi = gpu_grad(torch_gpu, prob, relaxed=True)
    ref = oracle.bptt(prob.W_rec, prob.W_in, prob.x, prob.target, prob.theta, prob.leak, prob.reset, prob.slope,
                      relaxed=True)
    assert rel_err(gWr, ref.dW_rec) <= 1e-4 and rel_err(gWi, ref.dW_in) <= 1e-4
    eps = 1e-5
    Wr64, Wi64 = prob.W_rec.astype(np.float64), prob.W_in.astype(np.float64)
    for _ in range(8):
        i, j = g.integers(0, 64), g.integers(0, 64)
        P, M = Wr64.copy(), Wr64.copy()
        P[i, j] += eps
        M[i, j] -= eps
        lp = oracle.bptt(P, Wi64, prob.x, prob.target, relaxed=True).loss
        lm = oracle.bptt(M, Wi64, prob.x, prob.target, relaxed=True).loss
        fd = (lp - lm) / (2 * eps)
        scale = max(abs(fd), 1e-2 * np.abs(gWr).max())
        assert abs(gWr[i, j] - fd) <= 1e-3 * scale, (i, j, gWr[i, j], fd)


def test_bptt_full_size_trials_sample(torch_gpu, oracle):
    """N = 2048, 256 inputs, T = 200, checkpoint 50, on three of the 128
    trials (the gradient of a batch is the mean of per-trial gradients, so
    every trial's gradient is checked through a run of that trial alone)."""
    prob = wl.bptt_problem(5)
    picks = [0, 77, 127]
    counts, loss, gWr, gWi = gpu_grad(torch_gpu, prob, trials=picks)
    ref = oracle.bptt(prob.W_rec, prob.W_in, prob.x[:, picks], prob.target, prob.theta, prob.leak, prob.reset,
                      prob.slope)
    assert np.array_equal(counts, ref.counts)
    assert rel_err(gWr, ref.dW_rec) <= 1e-4, rel_err(gWr, ref.dW_rec)
    assert rel_err(gWi, ref.dW_in) <= 1e-4, rel_err(gWi, ref.dW_in)
