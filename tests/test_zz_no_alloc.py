"""sn_bptt_forward_noalloc (the BPTT forward with the library's own device
workspace, for callers that cannot allocate) against sn_bptt_forward with a
caller workspace, through the C ABI: identical spike counts on two calls in a
row, the second smaller, so whatever the first left in the shared buffer
cannot change the second; both forward modes; the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2305_02510_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_02510_amd import _lib
    from paper_2305_02510_amd.bptt import _bind
    return _bind(_lib.load())


def forward_both(lib, prob, relaxed):
    import torch
    from paper_2305_02510_amd.bptt import SnBpttDesc
    T, B, Nin = prob.x.shape
    N = prob.W_rec.shape[0]
    d = SnBpttDesc(N, Nin, B, T, prob.checkpoint, prob.theta, prob.leak, prob.reset, prob.slope, int(relaxed))
    nbytes = lib.sn_bptt_workspace_bytes(ctypes.byref(d))
    assert 0 < nbytes <= 64 << 20
    W = torch.tensor(np.concatenate([prob.W_rec, prob.W_in]), dtype=torch.float32, device="cuda")
    x = torch.tensor(prob.x, dtype=torch.float32, device="cuda")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ref = torch.empty(B, N, dtype=torch.float32, device="cuda")
    got = torch.full((B, N), -1.0, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    assert lib.sn_bptt_forward(ctypes.byref(d), W.data_ptr(), x.data_ptr(), ref.data_ptr(), ws.data_ptr(),
                               stream) == 0
    assert lib.sn_bptt_forward_noalloc(ctypes.byref(d), W.data_ptr(), x.data_ptr(), got.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("relaxed", [False, True])
def test_noalloc_forward_matches_workspace_forward(lib, relaxed):
    # first call: the larger problem; second: a smaller one over the buffer
    # the first left behind
    for seed, n, nin, trials, steps, ckpt in [(91, 256, 64, 40, 60, 16), (92, 96, 40, 9, 33, 7)]:
        prob = wl.bptt_problem(seed, n=n, n_in=nin, trials=trials, steps=steps, checkpoint=ckpt)
        got, ref = forward_both(lib, prob, relaxed)
        assert np.array_equal(got, ref), f"counts differ (n={n}, trials={trials}, relaxed={relaxed})"
        if not relaxed:
            assert ref.sum() > 0


def test_noalloc_forward_limit(lib):
    from paper_2305_02510_amd.bptt import SnBpttDesc
    d = SnBpttDesc(2048, 256, 128, 200, 50, 1.0, 0.0625, 0.0, 10.0, 0)  # needs several hundred MB
    assert lib.sn_bptt_workspace_bytes(ctypes.byref(d)) > 64 << 20
    dummy = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    assert lib.sn_bptt_forward_noalloc(ctypes.byref(d), dummy, dummy, dummy, None) == -5  # SN_ERANGE
    assert lib.sn_bptt_forward_noalloc(None, dummy, dummy, dummy, None) == -1             # SN_EINVAL
