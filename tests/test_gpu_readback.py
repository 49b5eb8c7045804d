"""Device-memory readbacks (sn_read_raster_device, sn_read_state_device)
against the host readbacks and the oracle: ragged N (the last 64-neuron group
partly filled, an odd number of 32-bit words), several trials, a window that
starts after step 0, a many-trial dense net, the empty window and the range
errors."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2305_02510_amd import workloads as wl  # noqa: E402
from test_gpu_parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    bits = np.unpackbits(words.view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :n]


@pytest.mark.parametrize("n,trials,path", [(130, 3, "step"), (100, 1, "persist"), (4000, 2, "auto")])
def test_device_readbacks_match(torch_gpu, oracle, n, trials, path):
    torch = torch_gpu
    from paper_2305_02510_amd import Network
    net = wl.random_small(41 + n, n=n, p=min(0.3, 12.0 / n), max_delay=6, steps=50, trials=trials)
    print(f"device readback: N={n} B={trials} path={path}", flush=True)
    g = Network.from_workload(net)
    g.set_path(path)
    g.run(net.steps)
    W32 = (n + 31) // 32
    words = torch.full((trials, net.steps - 7, W32), -1, dtype=torch.int32, device="cuda")
    V = torch.full((trials, n), float("nan"), dtype=torch.float32, device="cuda")
    ref = torch.full((trials, n), 255, dtype=torch.uint8, device="cuda")
    g.read_raster_device(7, words)  # enqueued behind the run, no wait in between
    g.read_state_device(V, ref)
    g.synchronize()
    host_words = g.read_raster_words(7, net.steps - 7)
    hV, href = g.read_state()
    full = g.read_raster(0, net.steps)
    g.close()
    got = words.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, host_words)
    assert np.array_equal(V.cpu().numpy(), hV) and np.array_equal(ref.cpu().numpy(), href)
    assert not (unpack(got, W32 * 32)[..., n:]).any(), "bits beyond N must be clear"
    assert_parity(net, oracle.run_sparse(net), full, hV, href, "host readback")
    assert np.array_equal(unpack(got, n), full[:, 7:])


def test_device_readback_dense_trials(torch_gpu):
    torch = torch_gpu
    from paper_2305_02510_amd import Network
    net = wl.dense_trials(3, n=200, trials=5, steps=30)
    g = Network.from_workload(net)
    g.run(net.steps)
    words = torch.zeros((5, 30, 7), dtype=torch.int32, device="cuda")
    g.read_raster_device(0, words)
    g.synchronize()
    assert np.array_equal(words.cpu().numpy().view(np.uint32), g.read_raster_words(0, 30))
    g.close()


def test_device_readback_edges(torch_gpu):
    torch = torch_gpu
    from paper_2305_02510_amd import Network
    from paper_2305_02510_amd._lib import SnError
    net = wl.random_small(5, n=70, steps=20)
    g = Network.from_workload(net)
    g.run(10)
    empty = torch.zeros((1, 0, 3), dtype=torch.int32, device="cuda")
    g.read_raster_device(10, empty)  # an empty window at the current step is fine
    with pytest.raises(SnError):
        g.read_raster_device(5, torch.zeros((1, 6, 3), dtype=torch.int32, device="cuda"))  # step 10 not simulated
    with pytest.raises(SnError):
        g.read_raster_device(-1, torch.zeros((1, 2, 3), dtype=torch.int32, device="cuda"))
    st = g.lib.sn_read_raster_device(g.h, 0, 2, None)
    assert st != 0  # NULL output
    g.read_state_device(None, None)  # nothing asked, nothing written
    g.synchronize()
    g.close()
