"""CPU oracle of the matrix-form LIF simulation with synaptic delays.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product (the HIP library and
its binding) never imports, links or runs anything here.

The computation lives in ``lif_oracle.c`` (plain C, double precision, one
thread); this module compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lif_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OR_OK = 0
OR_NONEXACT = -6


def build(src: str = SRC, out: str = LIB, extra_flags=()) -> str:
    """Compile the oracle (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-Wall", *extra_flags, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def _bind(lib):
    lib.or_lif_sparse.restype = ctypes.c_int
    lib.or_lif_sparse.argtypes = [_I32, _I32, _I32, _I32, _P, _P, _P, _P, _P,
                                  _I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int]
    lib.or_lif_sparse_driven.restype = ctypes.c_int
    lib.or_lif_sparse_driven.argtypes = [_I32, _I32, _I32, _I32, _P, _P, _P, _P, _P,
                                         _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int]
    lib.or_bptt.restype = ctypes.c_int
    lib.or_bptt.argtypes = [_I32, _I32, _I32, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.or_lif_stdp.restype = ctypes.c_int
    lib.or_lif_stdp.argtypes = [_I32, _I32, _I32, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P,
                                _I32, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.or_lif_columns.restype = ctypes.c_int
    lib.or_lif_columns.argtypes = [_I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P,
                                   _P, _P, _P, _P, _P, _P, ctypes.c_int]
    lib.or_lif_dense.restype = ctypes.c_int
    lib.or_lif_dense.argtypes = [_I32, _I32, _I32, _P, _P, _P, _P, _P,
                                 _P, _P, _P, _P, _P, ctypes.c_int]
    return lib


@dataclasses.dataclass
class OracleResult:
    spikes: np.ndarray      # uint8 [B][T][N]
    V: np.ndarray           # float64 [B][N], state after the last step
    ref: np.ndarray         # int32 [B][N], refractory steps left
    exact: bool             # every partial sum provably exact in binary32


class Oracle:
    def __init__(self, path: Optional[str] = None):
        path = path or LIB
        if not os.path.exists(path):
            build(out=path)
        self.lib = _bind(ctypes.CDLL(path))

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)

    def _params(self, net):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        return (f(net.threshold), f(net.leak), f(net.reset),
                np.ascontiguousarray(net.refractory, dtype=np.int32), f(net.amplitude))

    def run_sparse(self, net, steps: Optional[int] = None, trials=None) -> OracleResult:
        """Simulate ``net`` through its COO synapse list for ``steps`` steps
        (default: all), for all trials or the listed trial indices."""
        T = net.steps if steps is None else int(steps)
        ext = net.ext[:, :T] if trials is None else net.ext[list(trials), :T]
        ext = np.ascontiguousarray(ext, dtype=np.uint8)
        B, N = ext.shape[0], net.n
        th, lk, rs, rf, am = self._params(net)
        pre = np.ascontiguousarray(net.pre, dtype=np.int32)
        post = np.ascontiguousarray(net.post, dtype=np.int32)
        w = np.ascontiguousarray(net.weight, dtype=np.float64)
        d = np.ascontiguousarray(net.delay, dtype=np.int32)
        spikes = np.zeros((B, T, N), np.uint8)
        V = np.zeros((B, N), np.float64)
        ref = np.zeros((B, N), np.int32)
        P = self._ptr
        rc = self.lib.or_lif_sparse(N, B, int(net.max_delay), T, P(th), P(lk), P(rs), P(rf), P(am),
                                    pre.shape[0], P(pre), P(post), P(w), P(d),
                                    P(ext), P(spikes), P(V), P(ref), 1)
        if rc not in (OR_OK, OR_NONEXACT):
            raise ValueError(f"oracle rejected the input (status {rc})")
        return OracleResult(spikes, V, ref, rc == OR_OK)

    def run_sparse_driven(self, net, history, posts=None, steps: Optional[int] = None,
                          syn_index=None) -> OracleResult:
        """The update of ``net`` with source spikes taken from ``history``
        (uint8 [B][>= T][N], e.g. the network's own raster).  With ``posts``
        (an index array), only the synapses into those neurons are summed:
        their columns of the result are meaningful, the others are not.
        ``syn_index`` (indices into the synapse list, e.g. every synapse into
        a post range) selects the synapses directly instead."""
        T = net.steps if steps is None else int(steps)
        ext = np.ascontiguousarray(net.ext[:, :T], dtype=np.uint8)
        B, N = ext.shape[0], net.n
        hist = np.ascontiguousarray(np.asarray(history)[:, :T], dtype=np.uint8)
        assert hist.shape == (B, T, N)
        pre, post, w, d = net.pre, net.post, net.weight, net.delay
        if syn_index is not None:
            pre, post, w, d = pre[syn_index], post[syn_index], w[syn_index], d[syn_index]
        elif posts is not None:
            keep = np.zeros(N, bool)
            keep[np.asarray(posts)] = True
            sel = keep[post]
            pre, post, w, d = pre[sel], post[sel], w[sel], d[sel]
        th, lk, rs, rf, am = self._params(net)
        pre = np.ascontiguousarray(pre, dtype=np.int32)
        post = np.ascontiguousarray(post, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.int32)
        spikes = np.zeros((B, T, N), np.uint8)
        V = np.zeros((B, N), np.float64)
        ref = np.zeros((B, N), np.int32)
        P = self._ptr
        rc = self.lib.or_lif_sparse_driven(N, B, int(net.max_delay), T, P(th), P(lk), P(rs), P(rf), P(am),
                                           pre.shape[0], P(pre), P(post), P(w), P(d), P(hist),
                                           P(ext), P(spikes), P(V), P(ref), 1)
        if rc not in (OR_OK, OR_NONEXACT):
            raise ValueError(f"oracle rejected the input (status {rc})")
        return OracleResult(spikes, V, ref, rc == OR_OK)

    def run_dense(self, net, steps: Optional[int] = None, trials=None, W=None) -> OracleResult:
        """Simulate ``net`` through its dense weight matrix (delay 1): W, or
        ``net.dense_weight`` when W is None."""
        if W is None:
            W = net.dense_weight
        assert W is not None
        T = net.steps if steps is None else int(steps)
        ext = net.ext[:, :T] if trials is None else net.ext[list(trials), :T]
        ext = np.ascontiguousarray(ext, dtype=np.uint8)
        B, N = ext.shape[0], net.n
        th, lk, rs, rf, am = self._params(net)
        W = np.ascontiguousarray(W, dtype=np.float64)
        spikes = np.zeros((B, T, N), np.uint8)
        V = np.zeros((B, N), np.float64)
        ref = np.zeros((B, N), np.int32)
        P = self._ptr
        rc = self.lib.or_lif_dense(N, B, T, P(th), P(lk), P(rs), P(rf), P(am), P(W),
                                   P(ext), P(spikes), P(V), P(ref), 1)
        if rc not in (OR_OK, OR_NONEXACT):
            raise ValueError(f"oracle rejected the input (status {rc})")
        return OracleResult(spikes, V, ref, rc == OR_OK)


    def run_columns(self, net, posts, wcol, history, steps: Optional[int] = None) -> OracleResult:
        """Neurons ``posts`` of a dense delay-1 net, one at a time, driven by
        the spike history ``history`` (uint8 [B][>= T][N]) of the whole network;
        wcol [S][N] are the weight columns W[:, posts].  Returns spikes
        [B][T][S] and the final V / ref [B][S] of the listed neurons."""
        T = net.steps if steps is None else int(steps)
        ext = np.ascontiguousarray(net.ext[:, :T], dtype=np.uint8)
        B, N = ext.shape[0], net.n
        posts = np.ascontiguousarray(posts, dtype=np.int32)
        S = posts.shape[0]
        wcol = np.ascontiguousarray(wcol, dtype=np.float64)
        history = np.ascontiguousarray(np.asarray(history)[:, :T], dtype=np.uint8)
        assert wcol.shape == (S, N) and history.shape == (B, T, N)
        th, lk, rs, rf, am = self._params(net)
        spikes = np.zeros((B, T, S), np.uint8)
        V = np.zeros((B, S), np.float64)
        ref = np.zeros((B, S), np.int32)
        P = self._ptr
        rc = self.lib.or_lif_columns(N, B, T, S, P(posts), P(th), P(lk), P(rs), P(rf), P(am), P(wcol),
                                     P(history), P(ext), P(spikes), P(V), P(ref), 1)
        if rc not in (OR_OK, OR_NONEXACT):
            raise ValueError(f"oracle rejected the input (status {rc})")
        return OracleResult(spikes, V, ref, rc == OR_OK)


@dataclasses.dataclass
class StdpResult:
    spikes: np.ndarray      # uint8 [T][N]
    V: np.ndarray           # float64 [N]
    ref: np.ndarray         # int32 [N]
    weight: np.ndarray      # float64 [nnz], after the last step, input order
    exact: bool


def _stdp(self, net, window, ltp, ltd, w_min, w_max, steps=None) -> StdpResult:
    """One trial of ``net`` with the plasticity rule of or_lif_stdp; ltp and
    ltd are sequences of ``window`` amplitudes."""
    T = net.steps if steps is None else int(steps)
    ext = np.ascontiguousarray(net.ext[0, :T], dtype=np.uint8)
    N = net.n
    th, lk, rs, rf, am = self._params(net)
    pre = np.ascontiguousarray(net.pre, dtype=np.int32)
    post = np.ascontiguousarray(net.post, dtype=np.int32)
    w = np.array(net.weight, dtype=np.float64)
    d = np.ascontiguousarray(net.delay, dtype=np.int32)
    # entries past the window are never read; they hold a sentinel so that a
    # rule reading past its window changes the result
    lp = np.full(16, 0.5)
    lm = np.full(16, 0.5)
    lp[:window] = ltp[:window]
    lm[:window] = ltd[:window]
    spikes = np.zeros((T, N), np.uint8)
    V = np.zeros(N)
    ref = np.zeros(N, np.int32)
    P = self._ptr
    rc = self.lib.or_lif_stdp(N, int(net.max_delay), T, P(th), P(lk), P(rs), P(rf), P(am), pre.shape[0], P(pre),
                              P(post), P(w), P(d), P(ext), P(spikes), P(V), P(ref), int(window), P(lp), P(lm),
                              float(w_min), float(w_max), 1)
    if rc not in (OR_OK, OR_NONEXACT):
        raise ValueError(f"oracle rejected the input (status {rc})")
    return StdpResult(spikes, V, ref, w, rc == OR_OK)


Oracle.stdp = _stdp


@dataclasses.dataclass
class BpttResult:
    loss: float
    dW_rec: np.ndarray   # float64 [N][N]
    dW_in: np.ndarray    # float64 [Nin][N]
    counts: np.ndarray   # float64 [B][N] spike counts


def _bptt(self, W_rec, W_in, x, target, theta=1.0, leak=0.0625, reset=0.0, slope=10.0, relaxed=False):
    """Surrogate-gradient BPTT of the recurrent LIF layer (see or_bptt).
    x: uint8 [T][B][Nin] input spikes."""
    W_rec = np.ascontiguousarray(W_rec, np.float64)
    W_in = np.ascontiguousarray(W_in, np.float64)
    x = np.ascontiguousarray(x, np.uint8)
    target = np.ascontiguousarray(target, np.float64)
    T, B, Nin = x.shape
    N = W_rec.shape[0]
    dWr = np.zeros((N, N))
    dWi = np.zeros((Nin, N))
    counts = np.zeros((B, N))
    loss = ctypes.c_double()
    P = self._ptr
    rc = self.lib.or_bptt(N, Nin, B, T, theta, leak, reset, slope, int(relaxed), P(W_rec), P(W_in), P(x),
                          P(target), ctypes.cast(ctypes.byref(loss), ctypes.c_void_p), P(dWr), P(dWi), P(counts))
    if rc != OR_OK:
        raise ValueError(f"oracle rejected the input (status {rc})")
    return BpttResult(loss.value, dWr, dWi, counts)


Oracle.bptt = _bptt

def host_workers() -> int:
    """Threads for fanning independent oracle runs (trials, nets, column
    chunks) out over the host's cores: the cores this process may use, at
    most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - non-Linux hosts
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def post_ranges(net, parts: int):
    """Splits the neurons of ``net`` into ``parts`` contiguous post ranges and
    returns [(j0, j1, syn_index)], syn_index = the synapses into [j0, j1)."""
    bounds = np.linspace(0, net.n, parts + 1).astype(np.int64)
    which = (np.searchsorted(bounds, net.post, side="right") - 1).astype(np.uint16)
    order = np.argsort(which, kind="stable")  # a radix sort for 16-bit keys
    cuts = np.searchsorted(which[order], np.arange(parts + 1), side="left")
    return [(int(bounds[r]), int(bounds[r + 1]), order[cuts[r]:cuts[r + 1]]) for r in range(parts)]


def fan_out(fn, items, workers: Optional[int] = None) -> list:
    """[fn(x) for x in items], the calls spread over host threads.  Each call
    is one single-threaded oracle run; ctypes releases the interpreter lock
    while the C code runs, so the calls proceed in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    items = list(items)
    w = max(1, min(workers or host_workers(), len(items) or 1))
    if w == 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(w) as ex:
        return list(ex.map(fn, items))


_default: Optional[Oracle] = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
