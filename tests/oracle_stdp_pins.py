"""Pins of the oracle's plasticity rule (or_lif_stdp) to closed forms and to a
second transcription of the rule.

The rule (chosen: §2.1 names STDP for the matrix mode without giving one): a
spike of i at tau arrives at j at tau + d; after the update of step t,
  - j spikes at t: the latest arrival t_a <= t with t - t_a < W adds ltp[t - t_a];
  - a spike of i arrives at t: the latest spike of j at t_post < t with
    t - t_post <= W subtracts ltd[t - t_post - 1];
  - the weight is clipped to [w_min, w_max]; new weights act from step t + 1.
"""
from __future__ import annotations

import numpy as np

from oracle_pins import tiny_net
from paper_2305_02510_amd.workloads import random_small

LTP = [16 / 64, 8 / 64, 4 / 64, 2 / 64, 1 / 64]
LTD = [12 / 64, 6 / 64, 3 / 64, 2 / 64, 1 / 64]
W = 5


def pair_net(t_pre, t_post, d, steps=40, w0=0.0):
    """Neuron 0 is kicked at t_pre, neuron 1 at t_post (amplitude 2 > threshold
    1, no refractory period); one synapse 0 -> 1 of weight w0, delay d."""
    return tiny_net(2, [0], [1], [w0], [d], steps=steps, refractory=0,
                    ext_events=[(0, t_pre, 0), (0, t_post, 1)], max_delay=max(d, 1))


def expected_pair(t_pre, t_post, d):
    arrival = t_pre + d
    lag = t_post - arrival
    if 0 <= lag < W:
        return LTP[lag]
    if -W <= lag < 0:
        return -LTD[-lag - 1]
    return 0.0


def pin_stdp_pair_closed_form(oracle):
    for d in (1, 2, 5):
        for t_pre in (3, 10):
            for t_post in range(0, 24):
                if t_post == t_pre:
                    continue
                net = pair_net(t_pre, t_post, d)
                res = oracle.stdp(net, W, LTP, LTD, -4.0, 4.0)
                want = expected_pair(t_pre, t_post, d)
                assert res.weight[0] == want, (d, t_pre, t_post, res.weight[0], want)


def pin_stdp_nearest_arrival(oracle):
    """Two arrivals before one post spike: only the latest counts."""
    net = tiny_net(2, [0], [1], [0.0], [2], steps=20, refractory=0,
                   ext_events=[(0, 3, 0), (0, 5, 0), (0, 9, 1)])
    res = oracle.stdp(net, W, LTP, LTD, -4.0, 4.0)
    # arrivals at 5 and 7; post spike at 9: LTP lag 2; arrival at 5 and 7 see no earlier post spike
    assert res.weight[0] == LTP[2]


def pin_stdp_window_edge(oracle):
    for lag in range(0, W + 2):
        net = tiny_net(2, [0], [1], [0.0], [1], steps=30, refractory=0,
                       ext_events=[(0, 4, 0), (0, 5 + lag, 1)])
        res = oracle.stdp(net, W, LTP, LTD, -4.0, 4.0)
        assert res.weight[0] == (LTP[lag] if lag < W else 0.0), lag
    for lag in range(1, W + 2):   # post spike lag steps before the arrival
        net = tiny_net(2, [0], [1], [0.0], [1], steps=30, refractory=0,
                       ext_events=[(0, 10, 1), (0, 9 + lag, 0)])
        res = oracle.stdp(net, W, LTP, LTD, -4.0, 4.0)
        assert res.weight[0] == (-LTD[lag - 1] if lag <= W else 0.0), lag


def pin_stdp_clip(oracle):
    net = pair_net(3, 5, 1, w0=0.125)
    res = oracle.stdp(net, W, LTP, LTD, -0.5, 0.25)
    assert res.weight[0] == 0.25           # 0.125 + 0.125 clipped at w_max
    net = pair_net(8, 8, 1, w0=-0.4375)    # arrival at 9, post spike at 8: depression ltd[0]
    res = oracle.stdp(net, W, LTP, LTD, -0.5, 0.25)
    assert res.weight[0] == -0.5           # -0.4375 - 0.1875 clipped at w_min


def pin_stdp_off_is_plain_simulation(oracle):
    for seed in range(3):
        net = random_small(700 + seed, n=16, p=0.3, max_delay=4, steps=50)
        res = oracle.stdp(net, 4, [0.0] * 4, [0.0] * 4, -8.0, 8.0)
        plain = oracle.run_sparse(net)
        assert np.array_equal(res.spikes, plain.spikes[0]) and np.array_equal(res.V, plain.V[0])
        assert np.array_equal(res.weight, net.weight.astype(np.float64))


def _transcribed_stdp(net, window, ltp, ltd, w_min, w_max):
    """The rule and the model written out again, one synapse and neuron at a
    time with plain Python floats."""
    n, T = net.n, net.steps
    w = [float(x) for x in net.weight]
    syn = list(zip(net.pre.tolist(), net.post.tolist(), net.delay.tolist()))
    V = [float(x) for x in net.reset]
    rho = [0] * n
    hist = []
    for t in range(T):
        U = []
        for j in range(n):
            u, r = V[j], float(net.reset[j])
            u = max(u - float(net.leak[j]), r) if u > r else (min(u + float(net.leak[j]), r) if u < r else u)
            U.append(u)
        for k, (i, j, d) in enumerate(syn):
            if t - d >= 0 and hist[t - d][i]:
                U[j] += w[k]
        s_now = [0] * n
        for j in range(n):
            u = U[j] + (float(net.amplitude[j]) if net.ext[0, t, j] else 0.0)
            fire = u > float(net.threshold[j])
            if rho[j] > 0:
                rho[j] -= 1
                V[j] = u
            elif fire:
                s_now[j] = 1
                V[j], rho[j] = float(net.reset[j]), int(net.refractory[j])
            else:
                V[j] = u
        hist.append(s_now)
        for k, (i, j, d) in enumerate(syn):
            change = 0.0
            if s_now[j]:
                for lag in range(window):
                    tau = t - lag - d
                    if tau < 0:
                        break
                    if hist[tau][i]:
                        change += ltp[lag]
                        break
            if t - d >= 0 and hist[t - d][i]:
                for lag in range(1, window + 1):
                    if t - lag < 0:
                        break
                    if hist[t - lag][j]:
                        change -= ltd[lag - 1]
                        break
            w[k] = min(max(w[k] + change, w_min), w_max)
    return np.array(hist, np.uint8), np.array(V), np.array(rho), np.array(w)


def pin_stdp_transcription(oracle):
    for seed in range(4):
        net = random_small(800 + seed, n=10, p=0.4, max_delay=3, steps=45, drive_p=0.35)
        window = 3 + seed % 3
        sp, V, rho, w = _transcribed_stdp(net, window, LTP, LTD, -1.0, 1.5)
        res = oracle.stdp(net, window, LTP, LTD, -1.0, 1.5)
        assert np.array_equal(res.spikes, sp), f"seed {seed}"
        assert np.array_equal(res.V, V) and np.array_equal(res.ref, rho)
        assert np.array_equal(res.weight, w), f"weights, seed {seed}"


ALL_STDP_PINS = [pin_stdp_pair_closed_form, pin_stdp_nearest_arrival, pin_stdp_window_edge, pin_stdp_clip,
                 pin_stdp_off_is_plain_simulation, pin_stdp_transcription]
