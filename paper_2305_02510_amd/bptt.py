"""torch.autograd binding of the surrogate-gradient BPTT kernels (C ABI
sn_bptt_*): argument marshalling only; the forward, the recomputation from
checkpoints and the backward all run in the HIP library."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check


class SnBpttDesc(ctypes.Structure):
    _fields_ = [("n_neurons", ctypes.c_int32), ("n_inputs", ctypes.c_int32), ("n_trials", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("threshold", ctypes.c_float), ("leak", ctypes.c_float), ("reset", ctypes.c_float),
                ("slope", ctypes.c_float), ("relaxed", ctypes.c_int32)]


def _bind(lib):
    if getattr(lib, "_bptt_bound", False):
        return lib
    P = ctypes.c_void_p
    lib.sn_bptt_workspace_bytes.argtypes = [ctypes.POINTER(SnBpttDesc)]
    lib.sn_bptt_workspace_bytes.restype = ctypes.c_size_t
    lib.sn_bptt_forward.argtypes = [ctypes.POINTER(SnBpttDesc), P, P, P, P, P]
    lib.sn_bptt_forward.restype = ctypes.c_int32
    lib.sn_bptt_backward.argtypes = [ctypes.POINTER(SnBpttDesc), P, P, P, P, P, P]
    lib.sn_bptt_backward.restype = ctypes.c_int32
    lib.sn_bptt_forward_noalloc.argtypes = [ctypes.POINTER(SnBpttDesc), P, P, P, P]
    lib.sn_bptt_forward_noalloc.restype = ctypes.c_int32
    lib._bptt_bound = True
    return lib


class _LIFLayer(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W_cat, x, desc_tuple):
        lib = _bind(_lib.load())
        T, B, Nin = x.shape
        N = W_cat.shape[1]
        theta, leak, reset, slope, checkpoint, relaxed = desc_tuple
        d = SnBpttDesc(N, Nin, B, T, checkpoint, theta, leak, reset, slope, int(relaxed))
        nbytes = lib.sn_bptt_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise ValueError("invalid BPTT shape (N must be a positive multiple of 32)")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=W_cat.device)
        counts = torch.empty(B, N, dtype=torch.float32, device=W_cat.device)
        stream = torch.cuda.current_stream(W_cat.device).cuda_stream
        check(lib.sn_bptt_forward(ctypes.byref(d), W_cat.data_ptr(), x.data_ptr(), counts.data_ptr(),
                                  ws.data_ptr(), stream))
        ctx.desc = d
        ctx.save_for_backward(W_cat, x, ws)
        return counts

    @staticmethod
    def backward(ctx, dcounts):
        lib = _bind(_lib.load())
        W_cat, x, ws = ctx.saved_tensors
        dcounts = dcounts.contiguous().float()
        dW = torch.empty_like(W_cat)
        stream = torch.cuda.current_stream(W_cat.device).cuda_stream
        check(lib.sn_bptt_backward(ctypes.byref(ctx.desc), W_cat.data_ptr(), x.data_ptr(), dcounts.data_ptr(),
                                   ws.data_ptr(), dW.data_ptr(), stream))
        return dW, None, None


def spike_counts(W_rec: torch.Tensor, W_in: torch.Tensor, x: torch.Tensor, threshold: float = 1.0,
                 leak: float = 0.0625, reset: float = 0.0, slope: float = 10.0, checkpoint: int = 50,
                 relaxed: bool = False) -> torch.Tensor:
    """Spike counts [B][N] of the recurrent LIF layer over x [T][B][Nin]
    (float32 on the device), differentiable in W_rec and W_in through the
    fast-sigmoid surrogate."""
    W_cat = torch.cat([W_rec, W_in], 0).contiguous().float()
    x = x.contiguous().float()
    return _LIFLayer.apply(W_cat, x, (float(threshold), float(leak), float(reset), float(slope), int(checkpoint),
                                      bool(relaxed)))
