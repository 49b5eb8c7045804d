"""Seeded synthetic workloads for the LIF-with-delays simulation.

This module only *generates inputs*: network topology, weights, delays, neuron
parameters and external spike trains.  It holds none of the model's arithmetic
and imports neither the GPU binding nor the CPU oracle, so both consume exactly
the same arrays.

Random numbers come from numpy's Philox4x32-10 counter-based generator (Salmon
et al., SC'11), keyed per (seed, stream) through a SeedSequence, so a
(config, seed) pair always yields identical bytes on a given numpy version.

Values follow the paper's benchmark recipe (§3: Erdos-Renyi graphs, neuron =
node, synapse = edge, a few externally driven input neurons) and the sizes of
the workloads this package is measured on.  All weights, thresholds, leaks,
reset states and amplitudes are multiples of 2^-6, so every partial sum the
model forms is exact in binary32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GRID = 64.0  # values are k / 64

_STREAMS = {"edge": 1, "w": 2, "d": 3, "inp": 4, "sel": 5, "param": 6, "size": 7, "target": 8}


def rng_for(seed: int, stream: str, *extra: int) -> np.random.Generator:
    """Independent Philox stream for (seed, stream name, extra indices)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF,
                                 _STREAMS[stream], *[int(e) for e in extra]])
    return np.random.Generator(np.random.Philox(ss))


@dataclasses.dataclass
class Network:
    """One network (shared by ``trials`` independent trials) plus its inputs.

    Neuron parameters are per-neuron arrays (§2.1 holds them as vectors).
    Synapses are a COO list pre -> post with weight and integer delay >= 1.
    ``dense_weight`` (row = pre, column = post) is set for dense nets, whose
    synapses all have delay 1; ``pre/post/weight/delay`` then list its nonzeros.
    ``ext`` is the external spike raster, uint8 [trials][steps][n] of 0/1.
    """
    name: str
    n: int
    trials: int
    max_delay: int
    steps: int
    threshold: np.ndarray
    leak: np.ndarray
    reset: np.ndarray
    refractory: np.ndarray
    amplitude: np.ndarray
    pre: np.ndarray
    post: np.ndarray
    weight: np.ndarray
    delay: np.ndarray
    ext: np.ndarray
    dense_weight: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.pre.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.bincount(self.pre, minlength=self.n).astype(np.int64)

    def validate(self) -> None:
        n = self.n
        assert self.threshold.shape == (n,) and self.threshold.dtype == np.float32
        assert self.leak.shape == (n,) and self.leak.dtype == np.float32
        assert self.reset.shape == (n,) and self.reset.dtype == np.float32
        assert self.refractory.shape == (n,) and self.refractory.dtype == np.uint8
        assert self.amplitude.shape == (n,) and self.amplitude.dtype == np.float32
        assert self.pre.dtype == np.int32 and self.post.dtype == np.int32
        assert self.weight.dtype == np.float32 and self.delay.dtype == np.uint8
        assert self.ext.shape == (self.trials, self.steps, n) and self.ext.dtype == np.uint8
        if self.nnz:
            assert self.pre.min() >= 0 and self.pre.max() < n
            assert self.post.min() >= 0 and self.post.max() < n
            assert self.delay.min() >= 1 and self.delay.max() <= self.max_delay


def _params(n, theta, leak, reset, refractory, amplitude):
    def full(x, dt):
        a = np.asarray(x, dtype=dt)
        return np.ascontiguousarray(np.broadcast_to(a, (n,)).astype(dt))
    return (full(theta, np.float32), full(leak, np.float32), full(reset, np.float32),
            full(refractory, np.uint8), full(amplitude, np.float32))


def erdos_renyi_edges(n: int, p: float, rng: np.random.Generator,
                      n_pre: Optional[int] = None, n_post: Optional[int] = None):
    """Directed Erdos-Renyi edges without self-loops (§3 uses networkx's
    G(n, p)); every ordered pair (i, j), i != j, independently with prob. p.

    Pre-neurons range over [0, n_pre), post-neurons over [0, n_post) (both
    default to n).  Edges are drawn by geometric skipping over the pair index
    space, so the cost is O(edges), and come out sorted by (pre, post).
    """
    n_pre = n if n_pre is None else n_pre
    n_post = n if n_post is None else n_post
    if p <= 0.0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    # Pair index q enumerates (i, j) row-major over [0,n_pre) x [0,n_post);
    # self pairs are rejected afterwards.
    total = n_pre * n_post
    if p >= 1.0:
        q = np.arange(total, dtype=np.int64)
    else:
        chunks = []
        pos = -1
        expect = int(total * p + 10 * math.sqrt(total * p) + 64)
        while True:
            gaps = rng.geometric(p, size=max(expect, 1024)).astype(np.int64)
            cand = pos + np.cumsum(gaps)
            cand = cand[cand < total]
            if cand.size:
                chunks.append(cand)
                pos = int(cand[-1])
            if cand.size < gaps.size:
                break
            expect = max(1024, int((total - pos) * p * 1.1) + 64)
        q = np.concatenate(chunks) if chunks else np.zeros(0, np.int64)
    i = (q // n_post).astype(np.int32)
    j = (q % n_post).astype(np.int32)
    keep = i != j
    return np.ascontiguousarray(i[keep]), np.ascontiguousarray(j[keep])


def _dyadic_uniform(rng, lo_k: int, hi_k: int, size) -> np.ndarray:
    """k / 64 with integer k uniform in [lo_k, hi_k]."""
    return (rng.integers(lo_k, hi_k + 1, size=size).astype(np.float32) / np.float32(GRID))


def _bernoulli_raster(rng, shape, p) -> np.ndarray:
    return (rng.random(shape) < p).astype(np.uint8)


# --------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------

def single_lif(seed: int = 1, steps: int = 100) -> Network:
    """Small net: 100 LIF neurons plus 10 input neurons spiking Bernoulli(0.1)
    per step; random connectivity p = 0.1 from all 110 into the 100; weights
    k/64 with k uniform in [-64, 128] (w in [-1, 2]); delays uniform 1..3;
    threshold 1, reset 0, leak 2^-3, refractory 2; T = 100."""
    n_net, n_in = 100, 10
    n = n_net + n_in
    th, lk, rs, rf, am = _params(n, 1.0, 0.125, 0.0, 2, 2.0)
    rf[n_net:] = 0
    g = rng_for(seed, "edge")
    mask = g.random((n, n_net)) < 0.1
    mask[np.arange(n_net), np.arange(n_net)] = False
    pre, post = np.nonzero(mask)
    pre = pre.astype(np.int32)
    post = post.astype(np.int32)
    w = _dyadic_uniform(rng_for(seed, "w"), -64, 128, pre.shape[0])
    d = rng_for(seed, "d").integers(1, 4, size=pre.shape[0]).astype(np.uint8)
    ext = np.zeros((1, steps, n), np.uint8)
    ext[0, :, n_net:] = _bernoulli_raster(rng_for(seed, "inp"), (steps, n_in), 0.1)
    return Network("single_lif_n110", n, 1, 3, steps, th, lk, rs, rf, am,
                   pre, post, w, d, ext)


def large_sparse(seed: int = 2, n: int = 10_000, p: float = 0.01, steps: int = 1000,
                 w_k=(-32, 64), max_delay: int = 16, drive_frac: float = 0.05,
                 drive_p: float = 0.05, name: Optional[str] = None) -> Network:
    """Large sparse net: directed ER p = 0.01 over N = 10,000 (about 1M
    synapses); weights k/64, k uniform in [-32, 64] (w in [-0.5, 1]); delays
    uniform 1..16; 5% of the neurons (first 5% of a seeded permutation)
    receive Bernoulli(0.05) external spikes of amplitude 2; threshold 1,
    reset 0, leak 2^-4, refractory 2; T = 1000."""
    th, lk, rs, rf, am = _params(n, 1.0, 0.0625, 0.0, 2, 2.0)
    pre, post = erdos_renyi_edges(n, p, rng_for(seed, "edge"))
    w = _dyadic_uniform(rng_for(seed, "w"), w_k[0], w_k[1], pre.shape[0])
    d = rng_for(seed, "d").integers(1, max_delay + 1, size=pre.shape[0]).astype(np.uint8)
    n_drive = int(round(drive_frac * n))
    driven = np.sort(rng_for(seed, "sel").permutation(n)[:n_drive])
    ext = np.zeros((1, steps, n), np.uint8)
    ext[0][:, driven] = _bernoulli_raster(rng_for(seed, "inp"), (steps, n_drive), drive_p)
    return Network(name or f"large_sparse_n{n}_p{p}", n, 1, max_delay, steps, th, lk, rs, rf, am,
                   pre, post, w, d, ext)


def large_sparse_xl(seed: int = 7, p: float = 0.01, **kw) -> Network:
    """The largest point of the size and sparsity grid the paper benchmarks
    (§3: ER nets of growing size and connection probability): N = 100,000 at
    p = 0.001 (about 1e7 synapses) or p = 0.01 (about 1e8), otherwise as
    large_sparse (weights k/64 in [-0.5, 1], delays 1..16, 5% of the neurons
    driven Bernoulli(0.05), threshold 1, reset 0, leak 2^-4, refractory 2,
    T = 1000)."""
    kw.setdefault("name", f"large_sparse_xl_n100000_p{p}")
    return large_sparse(seed, n=100_000, p=p, **kw)


def large_sparse_low(seed: int = 2, **kw) -> Network:
    """Large sparse net with inhibition-dominated weights (k in [-64, 32]):
    firing stays low, so the event-driven push delivery is exercised."""
    kw.setdefault("name", "large_sparse_low_n10000")
    return large_sparse(seed, w_k=(-64, 32), **kw)


def balanced_dense_weights(n: int, rng_w: np.random.Generator, rng_sel: np.random.Generator,
                           inh_frac: float = 0.2, sigma_exc: float = 2.0,
                           sigma_inh: float = 8.0, kmax: int = 16) -> np.ndarray:
    """Dense N x N weights, row = pre: a seeded 20% of the pre-neurons are
    inhibitory (all their weights <= 0).  |w| = min(kmax, round(|z| sigma)) / 64
    with z standard normal, sigma 2 (excitatory) or 8 (inhibitory); zero
    diagonal.  With kmax = 16 every weight lies in [-0.25, 0.25]."""
    inh = np.zeros(n, bool)
    inh[rng_sel.permutation(n)[: int(round(inh_frac * n))]] = True
    z = np.abs(rng_w.standard_normal((n, n), dtype=np.float64))
    sigma = np.where(inh, sigma_inh, sigma_exc)[:, None]
    k = np.minimum(kmax, np.rint(z * sigma))
    k = np.where(inh[:, None], -k, k)
    np.fill_diagonal(k, 0)
    return (k / GRID).astype(np.float32)


def dense_trials(seed: int = 3, n: int = 4096, trials: int = 64, steps: int = 1000,
                 drive_p: float = 0.02) -> Network:
    """Large dense net, batched trials: fully connected N = 4096 (balanced
    excitatory/inhibitory weights in [-0.25, 0.25], 20% inhibitory), delay 1;
    64 independent trials sharing W, each neuron driven Bernoulli(0.02) per
    step with trial-specific streams, amplitude 2; threshold 1, reset 0,
    leak 2^-4, refractory 2; T = 1000."""
    th, lk, rs, rf, am = _params(n, 1.0, 0.0625, 0.0, 2, 2.0)
    W = balanced_dense_weights(n, rng_for(seed, "w"), rng_for(seed, "sel"))
    pre, post = np.nonzero(W)
    ext = np.empty((trials, steps, n), np.uint8)
    for b in range(trials):
        ext[b] = _bernoulli_raster(rng_for(seed, "inp", b), (steps, n), drive_p)
    return Network(f"dense_trials_n{n}_b{trials}", n, trials, 1, steps, th, lk, rs, rf, am,
                   pre.astype(np.int32), post.astype(np.int32), W[pre, post].copy(),
                   np.ones(pre.shape[0], np.uint8), ext, dense_weight=W)


def uneven_batch(seed: int = 4, count: int = 512, steps: int = 500,
                 n_range=(50, 5000), p_range=(0.005, 0.2)) -> List[Network]:
    """Uneven batch: independent nets with N log-uniform in [50, 5000],
    connection probability uniform in [0.005, 0.2], per-net maximum delay D
    uniform in 1..16 with per-synapse delays uniform in 1..D, per-net
    thresholds k/64 (k in [32, 128]) and leaks k/64 (k in [0, 8]); weights k/64
    with k in [-64, 64]; 5% of neurons driven Bernoulli(0.05); refractory 2;
    T = 500."""
    g = rng_for(seed, "size")
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    sizes = np.rint(np.exp(g.uniform(lo, hi, size=count))).astype(np.int64)
    probs = g.uniform(p_range[0], p_range[1], size=count)
    dmax = g.integers(1, 17, size=count)
    th_k = g.integers(32, 129, size=count)
    lk_k = g.integers(0, 9, size=count)
    nets = []
    for k in range(count):
        n = int(sizes[k])
        th, lk, rs, rf, am = _params(n, th_k[k] / GRID, lk_k[k] / GRID, 0.0, 2, 2.0)
        pre, post = erdos_renyi_edges(n, float(probs[k]), rng_for(seed, "edge", k))
        w = _dyadic_uniform(rng_for(seed, "w", k), -64, 64, pre.shape[0])
        D = int(dmax[k])
        d = rng_for(seed, "d", k).integers(1, D + 1, size=pre.shape[0]).astype(np.uint8)
        n_drive = max(1, int(round(0.05 * n)))
        driven = np.sort(rng_for(seed, "sel", k).permutation(n)[:n_drive])
        ext = np.zeros((1, steps, n), np.uint8)
        ext[0][:, driven] = _bernoulli_raster(rng_for(seed, "inp", k), (steps, n_drive), 0.05)
        nets.append(Network(f"uneven_{k}_n{n}", n, 1, D, steps, th, lk, rs, rf, am,
                            pre, post, w, d, ext))
    return nets


def random_small(seed: int, n: int = 12, p: float = 0.3, max_delay: int = 4,
                 steps: int = 40, trials: int = 1, w_k=(-64, 96), drive_p: float = 0.2,
                 hetero: bool = True) -> Network:
    """Tiny random net for exhaustive checks: heterogeneous dyadic parameters,
    random delays, self-loops and duplicate synapses included."""
    g = rng_for(seed, "param")
    if hetero:
        th = (g.integers(0, 129, size=n) / GRID).astype(np.float32)
        lk = (g.integers(0, 17, size=n) / GRID).astype(np.float32)
        rs = (g.integers(-32, 33, size=n) / GRID).astype(np.float32)
        rf = g.integers(0, 4, size=n).astype(np.uint8)
        am = (g.integers(-32, 193, size=n) / GRID).astype(np.float32)
    else:
        th, lk, rs, rf, am = _params(n, 1.0, 0.0625, 0.0, 2, 2.0)
    ge = rng_for(seed, "edge")
    mask = ge.random((n, n)) < p
    pre, post = np.nonzero(mask)
    # a few duplicates (summed by the model)
    dup = ge.random(pre.shape[0]) < 0.1
    pre = np.concatenate([pre, pre[dup]]).astype(np.int32)
    post = np.concatenate([post, post[dup]]).astype(np.int32)
    w = _dyadic_uniform(rng_for(seed, "w"), w_k[0], w_k[1], pre.shape[0])
    d = rng_for(seed, "d").integers(1, max_delay + 1, size=pre.shape[0]).astype(np.uint8)
    ext = _bernoulli_raster(rng_for(seed, "inp"), (trials, steps, n), drive_p)
    return Network(f"random_small_{seed}", n, trials, max_delay, steps, th, lk, rs, rf, am,
                   pre, post, w, d, ext)


def paper_table_shape(seed: int, n: int, p: float, steps: int = 1000) -> Network:
    """The benchmark networks of the paper's results section: ER graph of n
    neurons with connection probability p, 1000 steps, 3 random input neurons
    each spiked externally every 10 steps; threshold 1, reset 0, refractory 0,
    all weights 1 and delays 1.  The paper does not state the external spike
    amplitude or the leak; amplitude 2 (so a lone external spike fires a
    resting neuron) and leak 0 are used."""
    th, lk, rs, rf, am = _params(n, 1.0, 0.0, 0.0, 0, 2.0)
    pre, post = erdos_renyi_edges(n, p, rng_for(seed, "edge"))
    w = np.ones(pre.shape[0], np.float32)
    d = np.ones(pre.shape[0], np.uint8)
    inputs = np.sort(rng_for(seed, "sel").permutation(n)[:3])
    ext = np.zeros((1, steps, n), np.uint8)
    ext[0, ::10, :][:, inputs] = 1
    return Network(f"paper_table_n{n}_p{p}", n, 1, 1, steps, th, lk, rs, rf, am,
                   pre, post, w, d, ext)


ROW_BLOCK = 256  # rows of a dense-rows net drawn from one Philox stream


def _byte_table(counts) -> np.ndarray:
    """256-entry table mapping a uniform byte to k: value k fills counts[k]
    consecutive entries (counts sum to 256), so P(k) = counts[k] / 256."""
    table = np.concatenate([np.full(c, k, np.int8) for k, c in sorted(counts.items())])
    assert table.shape == (256,)
    return table


@dataclasses.dataclass
class RowsNetwork:
    """A dense delay-1 net too large to hold its weights as one array:
    W = k * 2^-e (row = pre, column = post) with int8 numerators drawn on
    demand, ROW_BLOCK rows per Philox stream, so any block of rows is
    reproducible on its own.  Pre-neuron i is inhibitory (row i <= 0) or
    excitatory (row i >= 0); within a row every entry is an independent byte
    mapped through the row type's table; the diagonal is zero.  ``ext`` is the
    external spike raster, uint8 [trials][steps][n] of 0/1."""
    name: str
    n: int
    trials: int
    steps: int
    e: int
    seed: int
    threshold: np.ndarray
    leak: np.ndarray
    reset: np.ndarray
    refractory: np.ndarray
    amplitude: np.ndarray
    inhibitory: np.ndarray  # bool [n]
    table_exc: np.ndarray   # int8 [256]
    table_inh: np.ndarray   # int8 [256]
    ext: np.ndarray

    def block(self, bi: int) -> np.ndarray:
        """Rows bi * ROW_BLOCK .. of k, int8 [rows][n]."""
        r0 = bi * ROW_BLOCK
        r1 = min(self.n, r0 + ROW_BLOCK)
        rows = r1 - r0
        raw = rng_for(self.seed, "w", bi).bit_generator.random_raw((rows * self.n + 7) // 8)
        u = raw.view(np.uint8)[: rows * self.n].reshape(rows, self.n)
        k = np.empty((rows, self.n), np.int8)
        for r in range(rows):
            np.take(self.table_inh if self.inhibitory[r0 + r] else self.table_exc, u[r], out=k[r])
            k[r, r0 + r] = 0
        return k

    @property
    def n_blocks(self) -> int:
        return (self.n + ROW_BLOCK - 1) // ROW_BLOCK

    @property
    def block_rows(self) -> int:
        return ROW_BLOCK

    def rows(self, r0: int, r1: int) -> np.ndarray:
        """Rows r0 .. r1 - 1 of k."""
        out = np.empty((r1 - r0, self.n), np.int8)
        for bi in range(r0 // ROW_BLOCK, (r1 + ROW_BLOCK - 1) // ROW_BLOCK):
            k = self.block(bi)
            a, b = max(r0, bi * ROW_BLOCK), min(r1, bi * ROW_BLOCK + k.shape[0])
            out[a - r0:b - r0] = k[a - bi * ROW_BLOCK:b - bi * ROW_BLOCK]
        return out

    def dense(self) -> np.ndarray:
        """All of W as float32 (small nets only)."""
        return (self.rows(0, self.n).astype(np.float32) * np.float32(2.0 ** -self.e))


def paper_scale_dense(seed: int = 6, n: int = 100_000, trials: int = 1, steps: int = 1000,
                      exc=None, inh=None, inh_frac: float = 0.2, drive_frac: float = 1.0,
                      drive_p: float = 0.02, leak: float = 0.25) -> RowsNetwork:
    """The paper's largest run (§4: 100,000 neurons, all-to-all, matrix mode)
    as a synthetic dense delay-1 net.  The paper states neither weights nor
    steps.  Here W = k / 64 with 20% inhibitory pre-neurons and byte-table
    distributions balanced on average (``exc``: k = 1 with probability 1/4,
    else 0; ``inh``: k = -1), so the input of a neuron has mean about zero and
    a spread that grows with the number of spiking neurons; every neuron is
    driven Bernoulli(0.02) per step with amplitude 2 (as the dense-trials
    net); threshold 1, reset 0, leak 2^-2, refractory 2; T = 1000.  At
    N = 100,000 the rate swings between about 0.5% and 7% per step."""
    th, lk, rs, rf, am = _params(n, 1.0, leak, 0.0, 2, 2.0)
    inh_mask = np.zeros(n, bool)
    inh_mask[rng_for(seed, "sel").permutation(n)[: int(round(inh_frac * n))]] = True
    t_exc = _byte_table(exc if exc is not None else {0: 192, 1: 64})
    t_inh = _byte_table(inh if inh is not None else {-1: 256})
    driven = np.zeros(n, bool)
    driven[rng_for(seed, "sel", 1).permutation(n)[: int(round(drive_frac * n))]] = True
    ext = np.empty((trials, steps, n), np.uint8)
    for b in range(trials):
        ext[b] = _bernoulli_raster(rng_for(seed, "inp", b), (steps, n), drive_p) * driven
    return RowsNetwork(f"paper_scale_dense_n{n}", n, trials, steps, 6, seed, th, lk, rs, rf, am,
                       inh_mask, t_exc, t_inh, ext)


def by_name(name: str, seed: Optional[int] = None) -> Network:
    table = {
        "single_lif": (single_lif, 1),
        "large_sparse": (large_sparse, 2),
        "large_sparse_low": (large_sparse_low, 2),
        "dense_trials": (dense_trials, 3),
        "large_sparse_xl_p0.001": (lambda seed: large_sparse_xl(seed, p=0.001), 7),
        "large_sparse_xl_p0.01": (lambda seed: large_sparse_xl(seed, p=0.01), 7),
    }
    fn, default_seed = table[name]
    return fn(default_seed if seed is None else seed)


@dataclasses.dataclass
class BpttProblem:
    """Recurrent LIF layer training problem: weights, input spikes, target rates."""
    W_rec: np.ndarray     # float32 [N][N], dyadic
    W_in: np.ndarray      # float32 [Nin][N], dyadic
    x: np.ndarray         # uint8 [T][B][Nin]
    target: np.ndarray    # float32 [N]
    theta: float = 1.0
    leak: float = 0.0625
    reset: float = 0.0
    slope: float = 10.0
    checkpoint: int = 50

    @property
    def shape(self):
        T, B, Nin = self.x.shape
        return self.W_rec.shape[0], Nin, B, T


def bptt_problem(seed: int = 5, n: int = 2048, n_in: int = 256, trials: int = 128, steps: int = 200,
                 in_k=(0, 8), drive_p: float = 0.05, checkpoint: int = 50) -> BpttProblem:
    """Surrogate-gradient training workload: recurrent N = 2048 with the
    balanced dense weights of the dense-trials net (dyadic, |w| <= 0.25,
    delay 1), 256 input sources spiking Bernoulli(0.05) into the layer through
    W_in = k/64 (k uniform in [0, 8]), 128 trials, T = 200, target rates
    uniform in [0, 0.2], checkpoint every 50 steps; threshold 1, reset 0,
    leak 2^-4, no refractory period, surrogate slope 10."""
    W_rec = balanced_dense_weights(n, rng_for(seed, "w"), rng_for(seed, "sel"))
    W_in = _dyadic_uniform(rng_for(seed, "w", 1), in_k[0], in_k[1], (n_in, n)).astype(np.float32)
    x = _bernoulli_raster(rng_for(seed, "inp"), (steps, trials, n_in), drive_p)
    target = rng_for(seed, "target").uniform(0.0, 0.2, size=n).astype(np.float32)
    return BpttProblem(W_rec, W_in, x, target, checkpoint=checkpoint)
