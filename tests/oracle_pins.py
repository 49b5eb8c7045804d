"""Pins of the CPU oracle to facts fixed by the paper's model and by mathematics.

Every function takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with a closed form, an invariant, or the paper's own second
formulation of synaptic delay.  The same functions run against the real oracle
(``test_oracle_pins.py``) and against deliberately broken copies of it
(``test_oracle_mutants.py``), which must each fail at least one pin.

Model (§2.1 of the paper, with the readings listed in the oracle's header):
leak towards r without crossing it, then delayed input s(t-d) W, then external
spikes a x(t), spike if U > theta, refractory masking, reset to r.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2305_02510_amd.workloads import Network, random_small


def tiny_net(n, pre=(), post=(), w=(), d=(), *, steps, theta=1.0, leak=0.0, reset=0.0,
             refractory=0, amplitude=2.0, ext_events=(), trials=1, max_delay=None):
    """Hand-built network.  ext_events: iterable of (trial, t, neuron)."""
    full = lambda x, dt: np.ascontiguousarray(np.broadcast_to(np.asarray(x, dt), (n,)).astype(dt))
    ext = np.zeros((trials, steps, n), np.uint8)
    for (b, t, j) in ext_events:
        if t < steps:
            ext[b, t, j] = 1
    d = np.asarray(d, np.uint8)
    D = max_delay if max_delay is not None else (int(d.max()) if d.size else 1)
    return Network("tiny", n, trials, D, steps, full(theta, np.float32), full(leak, np.float32),
                   full(reset, np.float32), full(refractory, np.uint8), full(amplitude, np.float32),
                   np.asarray(pre, np.int32), np.asarray(post, np.int32),
                   np.asarray(w, np.float32), d, ext)


def spike_times(raster_bt_n, j):
    return list(np.nonzero(raster_bt_n[:, j])[0])


# ---------------------------------------------------------------------------
# P1: constant drive of one neuron (leak, threshold, reset, refractory).
# After a reset the state after m driven steps is r + m a - (m-1) lam (a > lam),
# first exceeding theta at k* = floor((theta - r - lam)/(a - lam)) + 1; the
# refractory window only masks spikes, so the period is max(k*, R + 1).
# ---------------------------------------------------------------------------

def constant_drive_expected(theta, lam, a, R, r, T):
    if a <= lam:
        # the state returns to r every step before the drive: U == r + a
        if r + a > theta:
            return list(range(0, T, R + 1))
        return []
    x = (theta - r - lam) / (a - lam)
    kstar = math.floor(x) + 1 if x >= 0 else 1
    period = max(kstar, R + 1)
    return list(range(kstar - 1, T, period))


CONSTANT_DRIVE_CASES = [
    # theta, lam, a, R, r
    (1.0, 0.125, 0.25, 0, 0.0),
    (1.0, 0.125, 0.25, 9, 0.0),
    (1.0, 0.125, 0.25, 7, 0.0),
    (1.0, 0.0, 0.25, 0, 0.0),       # exact tie at k = 4: U = 1.0 does not fire
    (1.0, 0.0, 0.25, 2, 0.0),
    (0.5, 0.25, 0.375, 1, -0.5),
    (3.0, 0.125, 0.5, 3, 0.25),
    (1.0, 0.25, 0.125, 0, 0.0),     # a <= lam: never fires
    (1.0, 0.25, 0.25, 0, 0.0),      # a == lam
    (0.5, 0.5, 1.0, 2, 0.0),        # a > theta: fires every R + 1
    (1.0, 0.0625, 2.0, 2, 0.0),
    (0.75, 0.125, 0.1875, 5, -0.25),
]


def pin_constant_drive(oracle):
    T = 64
    for (theta, lam, a, R, r) in CONSTANT_DRIVE_CASES:
        net = tiny_net(1, steps=T, theta=theta, leak=lam, reset=r, refractory=R, amplitude=a,
                       ext_events=[(0, t, 0) for t in range(T)])
        res = oracle.run_sparse(net)
        got = spike_times(res.spikes[0], 0)
        exp = constant_drive_expected(theta, lam, a, R, r, T)
        assert got == exp, f"constant drive {(theta, lam, a, R, r)}: {got[:6]} != {exp[:6]}"


# ---------------------------------------------------------------------------
# P1b: free relaxation towards the reset state after a single kick of
# amplitude a at t = 0: V(t) = r + a -/+ t lam, clamped at r.
# ---------------------------------------------------------------------------

def pin_leak_relaxation(oracle):
    for (a, lam, r) in [(-0.75, 0.125, 0.0), (0.75, 0.125, 0.0), (-1.0, 0.1875, 0.5),
                        (0.5, 0.0625, -0.25), (0.25, 0.0, 0.0), (-0.5, 0.25, 0.0)]:
        for T in range(1, 12):
            net = tiny_net(1, steps=T, theta=10.0, leak=lam, reset=r, amplitude=a,
                           ext_events=[(0, 0, 0)])
            res = oracle.run_sparse(net)
            k = T - 1
            exp = min(r + a + k * lam, r) if a < 0 else max(r + a - k * lam, r)
            assert res.V[0, 0] == exp, f"relaxation a={a} lam={lam} r={r} T={T}: {res.V[0,0]} != {exp}"
            assert not res.spikes.any()


# ---------------------------------------------------------------------------
# P2: one synapse 0 -> 1 of delay d.  A kick fires neuron 0 at t0; neuron 1
# receives w at exactly t0 + d, and fires iff w > theta (a tie does not fire).
# ---------------------------------------------------------------------------

def pin_single_delay(oracle):
    t0 = 3
    for d in (1, 2, 3, 5, 8, 16):
        for (w, fires) in [(1.5, True), (1.0, False), (0.75, False)]:
            T = t0 + d + 4
            net = tiny_net(2, [0], [1], [w], [d], steps=T, leak=0.0, ext_events=[(0, t0, 0)],
                           max_delay=16)
            res = oracle.run_sparse(net)
            assert spike_times(res.spikes[0], 0) == [t0], "kicked neuron must fire once"
            assert spike_times(res.spikes[0], 1) == ([t0 + d] if fires else [])
            assert res.V[0, 1] == (0.0 if fires else w)
            # one step before arrival the post-neuron is still at rest
            res2 = oracle.run_sparse(net, steps=t0 + d)
            assert res2.V[0, 1] == 0.0 and not res2.spikes[0, :, 1].any()


# ---------------------------------------------------------------------------
# P3: a chain 0 -> 1 -> ... -> m of supra-threshold synapses fires neuron k at
# t0 plus the sum of the first k delays.
# ---------------------------------------------------------------------------

def pin_chain(oracle):
    for delays in [(1, 1, 1), (2, 3, 1, 4), (5, 1, 7), (16, 16)]:
        m = len(delays)
        t0 = 2
        T = t0 + sum(delays) + 3
        net = tiny_net(m + 1, list(range(m)), list(range(1, m + 1)), [1.25] * m, list(delays),
                       steps=T, leak=0.125, ext_events=[(0, t0, 0)], max_delay=16)
        res = oracle.run_sparse(net)
        acc = t0
        for k in range(m + 1):
            assert spike_times(res.spikes[0], k) == [acc], f"chain {delays} neuron {k}"
            if k < m:
                acc += delays[k]


# ---------------------------------------------------------------------------
# P4: a two-neuron loop with delays d1, d2 oscillates with period d1 + d2 for
# the whole run (exercises the wrap of any delay ring).
# ---------------------------------------------------------------------------

def pin_loop(oracle):
    for (d1, d2, R) in [(1, 1, 1), (2, 5, 3), (16, 3, 0), (7, 7, 13)]:
        T = 150
        t0 = 1
        net = tiny_net(2, [0, 1], [1, 0], [1.5, 1.5], [d1, d2], steps=T, leak=0.0625,
                       refractory=R, ext_events=[(0, t0, 0)], max_delay=16)
        res = oracle.run_sparse(net)
        P = d1 + d2
        assert spike_times(res.spikes[0], 0) == list(range(t0, T, P))
        assert spike_times(res.spikes[0], 1) == list(range(t0 + d1, T, P))


# ---------------------------------------------------------------------------
# P5: refractoriness -- successive spikes of neuron j are >= R_j + 1 apart.
# ---------------------------------------------------------------------------

def check_refractory(spikes_btn, refractory):
    B, T, N = spikes_btn.shape
    for b in range(B):
        for j in range(N):
            ts = np.nonzero(spikes_btn[b, :, j])[0]
            if ts.size > 1:
                assert np.diff(ts).min() >= int(refractory[j]) + 1, f"refractory violated b={b} j={j}"


def pin_refractory(oracle):
    for seed in range(6):
        net = random_small(100 + seed, n=10, steps=60, drive_p=0.5)
        res = oracle.run_sparse(net)
        check_refractory(res.spikes, net.refractory)
        assert res.spikes.any()


# ---------------------------------------------------------------------------
# P6: the paper's own construction of delay (§2.1): a synapse of delay d is a
# chain of d-1 proxy neurons (threshold 0, infinite leak) joined by unit-delay
# synapses of weight 1, the last one carrying w.  Simulating the expanded
# unit-delay network must reproduce the original neurons exactly.
# ---------------------------------------------------------------------------

def proxy_expand(net: Network) -> Network:
    n = net.n
    pre, post, w = [], [], []
    extra = 0
    for (i, j, wk, dk) in zip(net.pre.tolist(), net.post.tolist(), net.weight.tolist(), net.delay.tolist()):
        src = i
        for _ in range(dk - 1):
            k = n + extra
            extra += 1
            pre.append(src); post.append(k); w.append(1.0)
            src = k
        pre.append(src); post.append(j); w.append(wk)
    m = n + extra
    cat = lambda a, v, dt: np.concatenate([a, np.full(extra, v, dt)]).astype(dt)
    ext = np.zeros((net.trials, net.steps, m), np.uint8)
    ext[:, :, :n] = net.ext
    return Network(net.name + "_proxy", m, net.trials, 1, net.steps,
                   cat(net.threshold, 0.0, np.float32), cat(net.leak, np.inf, np.float32),
                   cat(net.reset, 0.0, np.float32), cat(net.refractory, 0, np.uint8),
                   cat(net.amplitude, 0.0, np.float32),
                   np.asarray(pre, np.int32), np.asarray(post, np.int32), np.asarray(w, np.float32),
                   np.ones(len(pre), np.uint8), ext)


def pin_proxy_equivalence(oracle):
    for seed in range(8):
        net = random_small(200 + seed, n=9, p=0.35, max_delay=5, steps=50, trials=2, hetero=False)
        # proxies need a non-negative reset of 0 for the chain to relay; the
        # original neurons keep arbitrary parameters
        a = oracle.run_sparse(net)
        b = oracle.run_sparse(proxy_expand(net))
        assert np.array_equal(a.spikes, b.spikes[:, :, : net.n]), f"proxy raster seed {seed}"
        assert np.array_equal(a.V, b.V[:, : net.n]) and np.array_equal(a.ref, b.ref[:, : net.n])
    for seed in range(4):
        net = random_small(300 + seed, n=8, p=0.4, max_delay=4, steps=40, hetero=True)
        a = oracle.run_sparse(net)
        b = oracle.run_sparse(proxy_expand(net))
        assert np.array_equal(a.spikes, b.spikes[:, :, : net.n]), f"proxy raster hetero seed {seed}"
        assert np.array_equal(a.V, b.V[:, : net.n])


# ---------------------------------------------------------------------------
# P8: with no external input nothing ever spikes and V stays at r.
# ---------------------------------------------------------------------------

def pin_rest(oracle):
    for seed in range(3):
        net = random_small(400 + seed, n=12, steps=30)
        net.ext[:] = 0
        # a neuron whose threshold lies below its reset state fires at rest
        net.threshold[:] = np.maximum(net.threshold, net.reset)
        res = oracle.run_sparse(net)
        assert not res.spikes.any()
        assert np.array_equal(res.V[0], net.reset.astype(np.float64))


# ---------------------------------------------------------------------------
# P11: relabelling the neurons permutes the raster the same way.
# ---------------------------------------------------------------------------

def permute(net: Network, perm: np.ndarray) -> Network:
    inv = np.argsort(perm)      # old label i -> new label inv[i]
    return Network(net.name + "_perm", net.n, net.trials, net.max_delay, net.steps,
                   net.threshold[perm].copy(), net.leak[perm].copy(), net.reset[perm].copy(),
                   net.refractory[perm].copy(), net.amplitude[perm].copy(),
                   inv[net.pre].astype(np.int32), inv[net.post].astype(np.int32),
                   net.weight.copy(), net.delay.copy(), np.ascontiguousarray(net.ext[:, :, perm]))


def pin_permutation(oracle):
    for seed in range(4):
        net = random_small(500 + seed, n=11, steps=40, hetero=True)
        perm = np.random.default_rng(seed).permutation(net.n)
        a = oracle.run_sparse(net)
        b = oracle.run_sparse(permute(net, perm))
        assert np.array_equal(a.spikes[:, :, perm], b.spikes), f"permutation seed {seed}"
        assert np.array_equal(a.V[:, perm], b.V)


# ---------------------------------------------------------------------------
# P12: trials are independent: trial b of a batch equals a one-trial run.
# ---------------------------------------------------------------------------

def pin_trials(oracle):
    net = random_small(600, n=10, steps=40, trials=3, hetero=True)
    full = oracle.run_sparse(net)
    for b in range(3):
        one = oracle.run_sparse(net, trials=[b])
        assert np.array_equal(full.spikes[b], one.spikes[0]), f"trial {b}"
        assert np.array_equal(full.V[b], one.V[0]) and np.array_equal(full.ref[b], one.ref[0])


# ---------------------------------------------------------------------------
# Time invariance: delaying every external spike by s steps delays the raster
# by s steps (the state before any input is the rest state).
# ---------------------------------------------------------------------------

def pin_time_shift(oracle):
    for seed in range(3):
        net = random_small(700 + seed, n=10, steps=30, hetero=True)
        net.threshold[:] = np.maximum(net.threshold, net.reset)   # silent at rest
        s = 5 + seed
        shifted = Network(net.name, net.n, 1, net.max_delay, net.steps + s, net.threshold, net.leak,
                          net.reset, net.refractory, net.amplitude, net.pre, net.post, net.weight,
                          net.delay, np.concatenate([np.zeros((1, s, net.n), np.uint8), net.ext], 1))
        a = oracle.run_sparse(net)
        b = oracle.run_sparse(shifted)
        assert not b.spikes[:, :s].any()
        assert np.array_equal(a.spikes, b.spikes[:, s:]) and np.array_equal(a.V, b.V)


# ---------------------------------------------------------------------------
# Block-diagonal superposition: two disjoint nets simulated as one equal the
# two simulated apart.
# ---------------------------------------------------------------------------

def pin_disjoint_union(oracle):
    x = random_small(800, n=7, steps=35, hetero=True, max_delay=3)
    y = random_small(801, n=9, steps=35, hetero=True, max_delay=4)
    n = x.n + y.n
    cat = lambda a, b: np.concatenate([a, b])
    u = Network("union", n, 1, 4, 35, cat(x.threshold, y.threshold), cat(x.leak, y.leak),
                cat(x.reset, y.reset), cat(x.refractory, y.refractory), cat(x.amplitude, y.amplitude),
                cat(x.pre, y.pre + x.n).astype(np.int32), cat(x.post, y.post + x.n).astype(np.int32),
                cat(x.weight, y.weight), cat(x.delay, y.delay), np.concatenate([x.ext, y.ext], 2))
    ru, rx, ry = oracle.run_sparse(u), oracle.run_sparse(x), oracle.run_sparse(y)
    assert np.array_equal(ru.spikes[:, :, : x.n], rx.spikes)
    assert np.array_equal(ru.spikes[:, :, x.n:], ry.spikes)
    assert np.array_equal(ru.V[:, : x.n], rx.V) and np.array_equal(ru.V[:, x.n:], ry.V)


# ---------------------------------------------------------------------------
# Matrix form (§2.1, delay 1): U = leak(V) + s(t-1) W + a x(t) with numpy's
# matrix product, compared with the synapse-list oracle and the dense oracle.
# ---------------------------------------------------------------------------

def matrix_form(net: Network, W: np.ndarray):
    B, T, N = net.ext.shape
    th, lk, r = (net.threshold.astype(np.float64), net.leak.astype(np.float64),
                 net.reset.astype(np.float64))
    R = net.refractory.astype(np.int64)
    a = net.amplitude.astype(np.float64)
    spikes = np.zeros((B, T, N), np.uint8)
    V = np.tile(r, (B, 1))
    ref = np.zeros((B, N), np.int64)
    s_prev = np.zeros((B, N))
    for t in range(T):
        # clamped leak, vectorised
        U = np.where(V > r, np.maximum(V - lk, r), np.where(V < r, np.minimum(V + lk, r), V))
        U = U + s_prev @ W + a * net.ext[:, t, :]
        masked = ref > 0
        s = (U > th) & ~masked
        ref = np.where(masked, ref - 1, 0)
        ref = np.where(s, R, ref)
        V = np.where(s, r, U)
        spikes[:, t, :] = s
        s_prev = s.astype(np.float64)
    return spikes, V, ref


def pin_matrix_form(oracle):
    for seed in range(4):
        net = random_small(900 + seed, n=14, p=0.3, max_delay=1, steps=40, trials=2, hetero=True)
        W = np.zeros((net.n, net.n))
        np.add.at(W, (net.pre, net.post), net.weight.astype(np.float64))
        sp, V, ref = matrix_form(net, W)
        res = oracle.run_sparse(net)
        assert np.array_equal(res.spikes, sp), f"matrix form seed {seed}"
        assert np.array_equal(res.V, V) and np.array_equal(res.ref, ref)
        dense = Network(net.name, net.n, net.trials, 1, net.steps, net.threshold, net.leak, net.reset,
                        net.refractory, net.amplitude, net.pre, net.post, net.weight, net.delay,
                        net.ext, dense_weight=W.astype(np.float32))
        rd = oracle.run_dense(dense)
        assert np.array_equal(rd.spikes, sp) and np.array_equal(rd.V, V) and np.array_equal(rd.ref, ref)


# ---------------------------------------------------------------------------
# P13: brute force.  Every binary external input pattern of a 2- or 3-neuron
# net over a few steps, run as one trial each, against a second transcription
# of the six steps of the update (§2.1 with the readings above), written here
# independently of the oracle: plain Python floats, one neuron at a time.
# ---------------------------------------------------------------------------

def _transcribed_run(n, syn, theta, leak, reset, refr, amp, x):
    """x: [T][n] 0/1.  Returns (spikes [T][n], V [n], rho [n])."""
    V = [float(reset[j]) for j in range(n)]
    rho = [0] * n
    history = []
    for t in range(len(x)):
        s_now = [0] * n
        V_new = list(V)
        rho_new = list(rho)
        for j in range(n):
            U = V[j]
            if U > reset[j]:
                U = max(U - leak[j], reset[j])
            elif U < reset[j]:
                U = min(U + leak[j], reset[j])
            for (i, jj, w, d) in syn:
                if jj == j and t - d >= 0 and history[t - d][i]:
                    U += w
            U += amp[j] * x[t][j]
            fire = U > theta[j]
            if rho[j] > 0:
                s, rho_new[j] = 0, rho[j] - 1
            else:
                s, rho_new[j] = int(fire), 0
            if s:
                V_new[j], rho_new[j] = reset[j], int(refr[j])
            else:
                V_new[j] = U
            s_now[j] = s
        V, rho = V_new, rho_new
        history.append(s_now)
    return history, V, rho


def pin_brute_force(oracle):
    rng = np.random.default_rng(13)
    cases = [(2, 6, 1), (2, 6, 2), (3, 4, 1), (3, 4, 2), (2, 5, 2), (3, 4, 2)]
    for c, (n, T, D) in enumerate(cases):
        m = int(rng.integers(1, 6))
        pre = rng.integers(0, n, m)
        post = rng.integers(0, n, m)          # self-loops and duplicates allowed
        w = rng.choice([-1.0, -0.5, 0.25, 0.5, 1.0, 1.5], m)
        d = rng.integers(1, D + 1, m)
        theta = rng.choice([0.0, 0.5, 1.0], n)
        leak = rng.choice([0.0, 0.25, np.inf], n)
        reset = rng.choice([-0.5, 0.0, 0.25], n)
        theta = np.maximum(theta, reset)
        refr = rng.integers(0, 3, n)
        amp = rng.choice([0.5, 1.0, 2.0], n)
        B = 1 << (n * T)
        codes = np.arange(B, dtype=np.int64)
        ext = ((codes[:, None] >> np.arange(n * T)) & 1).astype(np.uint8).reshape(B, T, n)
        net = Network("brute", n, B, D, T, theta.astype(np.float32), leak.astype(np.float32),
                      reset.astype(np.float32), refr.astype(np.uint8), amp.astype(np.float32),
                      pre.astype(np.int32), post.astype(np.int32), w.astype(np.float32),
                      d.astype(np.uint8), ext)
        res = oracle.run_sparse(net)
        syn = list(zip(pre.tolist(), post.tolist(), w.tolist(), d.tolist()))
        for b in range(B):
            sp, V, rho = _transcribed_run(n, syn, theta.tolist(), leak.tolist(), reset.tolist(),
                                          refr.tolist(), amp.tolist(), ext[b].tolist())
            assert np.array_equal(res.spikes[b], np.asarray(sp, np.uint8)), f"brute force case {c} pattern {b}"
            assert np.array_equal(res.V[b], np.asarray(V)) and np.array_equal(res.ref[b], np.asarray(rho)), \
                f"brute force state, case {c} pattern {b}"


ALL_PINS = [pin_constant_drive, pin_leak_relaxation, pin_single_delay, pin_chain, pin_loop,
            pin_refractory, pin_proxy_equivalence, pin_rest, pin_permutation, pin_trials,
            pin_time_shift, pin_disjoint_union, pin_matrix_form, pin_brute_force]
