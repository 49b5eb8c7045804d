"""Python binding of the C ABI: argument marshalling only.

PyTorch supplies the device memory (its caching allocator, through the ABI's
allocator callbacks) and the stream (the current torch stream); every step of
the simulation runs in the HIP library.  There is no CPU fallback: if the
library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import check

PATHS = {"auto": _lib.PATH_AUTO, "small": _lib.PATH_SMALL, "step": _lib.PATH_STEP,
         "persist": _lib.PATH_PERSIST, "dense": _lib.PATH_DENSE, "push": _lib.PATH_PUSH,
         "dense_step": _lib.PATH_DENSE_STEP, "dense_rows": _lib.PATH_DENSE_ROWS}


class TorchAllocator:
    """sn_allocator backed by torch's caching allocator on one device."""

    def __init__(self, device):
        import torch
        self.device = device
        self.live = {}

        def _alloc(nbytes, _ctx):
            try:
                t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
            except Exception:  # out of memory: the library reports SN_ENOMEM
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, _ctx):
            self.live.pop(ptr, None)

        self._alloc = _lib.ALLOC_FN(_alloc)
        self._free = _lib.FREE_FN(_free)
        self.struct = _lib.SnAllocator(self._alloc, self._free, None)


def _f32(x, n):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, np.float32), (n,)))
    return a


def pack_bits(dense: np.ndarray) -> np.ndarray:
    """uint8 0/1 array [..., N] -> uint32 words [..., ceil(N/32)], bit j%32 of word j//32."""
    dense = np.asarray(dense, np.uint8)
    n = dense.shape[-1]
    w32 = (n + 31) // 32
    pad = np.zeros(dense.shape[:-1] + (w32 * 32,), np.uint8)
    pad[..., :n] = dense
    b = np.packbits(pad, axis=-1, bitorder="little")
    return np.ascontiguousarray(b).view(np.uint32).reshape(dense.shape[:-1] + (w32,))


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """Inverse of pack_bits."""
    words = np.ascontiguousarray(words, np.uint32)
    b = np.unpackbits(words.view(np.uint8), axis=-1, bitorder="little")
    return b[..., :n]


class Network:
    """A network of N LIF neurons x B trials on the current torch device."""

    def __init__(self, n: int, trials: int = 1, max_delay: int = 1, threshold=1.0, leak=0.0, reset=0.0,
                 refractory=0, amplitude=1.0, stream=None, use_torch_allocator: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the simulator runs only on the HIP device")
        self.lib = _lib.load()
        self.n, self.trials, self.max_delay = int(n), int(trials), int(max_delay)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._params = [_f32(threshold, n), _f32(leak, n), _f32(reset, n),
                        np.ascontiguousarray(np.broadcast_to(np.asarray(refractory, np.uint8), (n,))),
                        _f32(amplitude, n)]
        d = _lib.SnNetDesc()
        d.n_neurons, d.n_trials, d.max_delay = self.n, self.trials, self.max_delay
        d.threshold, d.leak, d.reset, d.refractory, d.amplitude = [p.ctypes.data for p in self._params]
        self._alloc = TorchAllocator(self.device) if use_torch_allocator else None
        handle = ctypes.c_void_p()
        check(self.lib.sn_create_network(ctypes.byref(d),
                                         ctypes.byref(self._alloc.struct) if self._alloc else None,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self.h = handle
        self.nnz = 0

    @classmethod
    def from_workload(cls, net, **kw) -> "Network":
        """Build from a workloads.Network (parameters, synapses and inputs)."""
        g = cls(net.n, net.trials, net.max_delay, net.threshold, net.leak, net.reset, net.refractory,
                net.amplitude, **kw)
        if net.dense_weight is not None:
            g.load_dense_weights(net.dense_weight)
        else:
            g.load_weights_delays(net.pre, net.post, net.weight, net.delay)
        g.set_input_spikes(0, net.ext)
        return g

    @classmethod
    def from_rows_workload(cls, net, posts=None, workers: int = 8, **kw):
        """Build from a workloads.RowsNetwork: its int8 row blocks are drawn
        in ``workers`` threads and loaded in order with sn_load_dense_rows_i8.
        Returns (network, cols): cols is int8 [len(posts)][N] = k[:, posts]
        when ``posts`` is given (columns for checking sampled neurons), else
        None.  ``network.out_degree`` holds the non-zero weights of every row."""
        from concurrent.futures import ThreadPoolExecutor
        g = cls(net.n, net.trials, 1, net.threshold, net.leak, net.reset, net.refractory, net.amplitude, **kw)
        posts = None if posts is None else np.asarray(posts, np.int64)
        cols = None if posts is None else np.empty((posts.shape[0], net.n), np.int8)
        g.out_degree = np.zeros(net.n, np.int64)
        window = max(1, 2 * workers)
        with ThreadPoolExecutor(max(1, workers)) as ex:
            for w0 in range(0, net.n_blocks, window):
                idx = range(w0, min(net.n_blocks, w0 + window))
                for bi, k in zip(idx, ex.map(net.block, idx)):
                    r0 = bi * net.block_rows
                    g.load_dense_rows_i8(r0, k, net.e)
                    g.out_degree[r0:r0 + k.shape[0]] = np.count_nonzero(k, axis=1)
                    if cols is not None:
                        cols[:, r0:r0 + k.shape[0]] = k[:, posts].T
        g.set_input_spikes(0, net.ext)
        return g, cols

    # -- loading -----------------------------------------------------------
    def load_weights_delays(self, pre, post, w, delay):
        pre = np.ascontiguousarray(pre, np.int32)
        post = np.ascontiguousarray(post, np.int32)
        w = np.ascontiguousarray(w, np.float32)
        delay = np.ascontiguousarray(delay, np.uint8)
        check(self.lib.sn_load_weights_delays(self.h, pre.shape[0], pre.ctypes.data, post.ctypes.data,
                                              w.ctypes.data, delay.ctypes.data))
        self.nnz = int(pre.shape[0])

    def load_dense_weights(self, W, delay: int = 1):
        W = np.ascontiguousarray(W, np.float32)
        assert W.shape == (self.n, self.n)
        check(self.lib.sn_load_dense_weights(self.h, W.ctypes.data, int(delay)))
        self.nnz = int(np.count_nonzero(W))

    def load_dense_rows_i8(self, row0: int, k, e: int):
        """Rows row0 .. row0 + len(k) - 1 of dense delay-1 weights W = k * 2^-e,
        k an int8 array [rows][N] (sn_load_dense_rows_i8)."""
        k = np.ascontiguousarray(k, np.int8)
        assert k.ndim == 2 and k.shape[1] == self.n
        check(self.lib.sn_load_dense_rows_i8(self.h, int(row0), int(k.shape[0]), k.ctypes.data, int(e)))
        self.nnz = 0

    def set_input_spikes(self, t0: int, spikes: np.ndarray):
        """spikes: uint8 0/1 [B][steps][N] or packed uint32 [B][steps][ceil(N/32)]."""
        spikes = np.asarray(spikes)
        if spikes.dtype != np.uint32:
            spikes = pack_bits(spikes)
        spikes = np.ascontiguousarray(spikes, np.uint32)
        assert spikes.ndim == 3 and spikes.shape[0] == self.trials
        check(self.lib.sn_set_input_spikes(self.h, int(t0), spikes.shape[1], spikes.ctypes.data))

    def set_input_spikes_device(self, t0: int, words) -> None:
        """words: torch int32/uint32 tensor on the device, [B][steps][ceil(N/32)]."""
        assert words.is_cuda and words.is_contiguous() and words.dim() == 3 and words.element_size() == 4
        assert words.shape[0] == self.trials and words.shape[2] == (self.n + 31) // 32
        check(self.lib.sn_set_input_spikes_device(self.h, int(t0), int(words.shape[1]), words.data_ptr()))

    # -- running -----------------------------------------------------------
    def set_path(self, path: str):
        check(self.lib.sn_set_path(self.h, PATHS[path]))

    def set_slices(self, slices: int):
        check(self.lib.sn_set_slices(self.h, int(slices)))

    def set_stdp(self, window: int, ltp, ltd, w_min: float, w_max: float):
        """Plasticity on (sn_set_stdp): ltp / ltd hold ``window`` amplitudes."""
        d = _lib.SnStdpDesc()
        d.window = int(window)
        for k in range(int(window)):
            d.ltp[k] = float(ltp[k])
            d.ltd[k] = float(ltd[k])
        d.w_min, d.w_max = float(w_min), float(w_max)
        check(self.lib.sn_set_stdp(self.h, ctypes.byref(d)))

    def stdp_off(self):
        check(self.lib.sn_set_stdp(self.h, None))

    def read_weights(self) -> np.ndarray:
        """Current weights in the order of the loaded synapse list."""
        w = np.zeros(self.nnz, np.float32)
        check(self.lib.sn_read_weights(self.h, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def autotune(self, steps: int = 64):
        """Times every strategy that can run this network over `steps` steps
        (sn_autotune) and keeps the fastest; resets the state.  Returns the
        chosen (path name, slice count; 0 = default plan)."""
        path, slices = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.sn_autotune(self.h, int(steps), ctypes.byref(path), ctypes.byref(slices)))
        return _lib.PATH_NAMES.get(path.value, str(path.value)), slices.value

    def run(self, steps: int):
        check(self.lib.sn_run(self.h, int(steps)))

    def synchronize(self):
        check(self.lib.sn_synchronize(self.h))

    def reset_state(self):
        check(self.lib.sn_reset_state(self.h))

    @property
    def progress(self):
        t = ctypes.c_int32()
        p = ctypes.c_int32()
        check(self.lib.sn_get_progress(self.h, ctypes.byref(t), ctypes.byref(p)))
        return t.value, _lib.PATH_NAMES.get(p.value, p.value)

    # -- reading -----------------------------------------------------------
    def read_raster_words(self, t0: int, steps: int) -> np.ndarray:
        out = np.zeros((self.trials, steps, (self.n + 31) // 32), np.uint32)
        check(self.lib.sn_read_raster(self.h, int(t0), int(steps), out.ctypes.data))
        return out

    def read_raster(self, t0: int, steps: int) -> np.ndarray:
        """uint8 0/1 spikes [B][steps][N]."""
        return unpack_bits(self.read_raster_words(t0, steps), self.n)

    def read_state(self):
        V = np.zeros((self.trials, self.n), np.float32)
        ref = np.zeros((self.trials, self.n), np.uint8)
        check(self.lib.sn_read_state(self.h, V.ctypes.data, ref.ctypes.data))
        return V, ref

    def read_raster_device(self, t0: int, out) -> None:
        """Spike words of steps t0 .. t0 + out.shape[1] - 1 into ``out``, a
        contiguous 4-byte integer tensor [B][steps][ceil(N/32)] on the
        network's device; asynchronous on the network's stream
        (sn_read_raster_device)."""
        assert out.is_cuda and out.is_contiguous() and out.dim() == 3 and out.element_size() == 4
        assert out.shape[0] == self.trials and out.shape[2] == (self.n + 31) // 32
        check(self.lib.sn_read_raster_device(self.h, int(t0), int(out.shape[1]), out.data_ptr()))

    def read_state_device(self, V=None, ref=None) -> None:
        """State into device tensors: V float32 [B][N], ref uint8 [B][N]
        (either may be None); asynchronous (sn_read_state_device)."""
        for x, dt in ((V, "torch.float32"), (ref, "torch.uint8")):
            if x is not None:
                assert x.is_cuda and x.is_contiguous() and str(x.dtype) == dt
                assert tuple(x.shape) == (self.trials, self.n)
        check(self.lib.sn_read_state_device(self.h, V.data_ptr() if V is not None else None,
                                            ref.data_ptr() if ref is not None else None))

    def close(self):
        if getattr(self, "h", None):
            self.lib.sn_destroy_network(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent networks advanced together by one persistent launch."""

    def __init__(self, networks):
        self.networks = list(networks)  # keeps the networks (and their allocators) alive
        self.lib = _lib.load()
        arr = (ctypes.c_void_p * len(self.networks))(*[g.h.value for g in self.networks])
        handle = ctypes.c_void_p()
        check(self.lib.sn_batch_create(arr, len(self.networks), ctypes.byref(handle)))
        self.h = handle

    def run(self, steps: int):
        check(self.lib.sn_batch_run(self.h, int(steps)))

    def autotune(self, steps: int = 64):
        """sn_batch_autotune: picks the fastest schedule over `steps` steps
        (every network is reset); returns (target_mult, team_share)."""
        tm, ts = ctypes.c_float(), ctypes.c_float()
        check(self.lib.sn_batch_autotune(self.h, int(steps), ctypes.byref(tm), ctypes.byref(ts)))
        return float(tm.value), float(ts.value)

    def synchronize(self):
        if self.networks:
            self.networks[0].synchronize()

    def close(self):
        if getattr(self, "h", None):
            self.lib.sn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
