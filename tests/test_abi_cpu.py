"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects malformed arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2305_02510_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "superneuro_mi.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sn_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_exports_every_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def _desc(n=10, b=1, d=1):
    d_ = _lib.SnNetDesc()
    d_.n_neurons, d_.n_trials, d_.max_delay = n, b, d
    d_.threshold_scalar, d_.leak_scalar, d_.amplitude_scalar = 1.0, 0.0, 1.0
    return d_


@pytest.mark.parametrize("n,b,d,code", [
    (0, 1, 1, _lib.SN_ERANGE), (-5, 1, 1, _lib.SN_ERANGE), ((1 << 20) + 1, 1, 1, _lib.SN_ERANGE),
    (10, 0, 1, _lib.SN_ERANGE), (10, 1, 0, _lib.SN_ERANGE), (10, 1, 65, _lib.SN_ERANGE),
])
def test_create_rejects_sizes(lib, n, b, d, code):
    out = ctypes.c_void_p()
    st = lib.sn_create_network(ctypes.byref(_desc(n, b, d)), None, None, ctypes.byref(out))
    assert st == code and not out.value
    assert lib.sn_last_error()


def test_create_rejects_bad_parameters(lib):
    out = ctypes.c_void_p()
    d = _desc()
    d.leak_scalar = -0.5
    assert lib.sn_create_network(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.SN_EINVAL
    assert b"leak" in lib.sn_last_error()
    d = _desc()
    d.threshold_scalar = float("nan")
    assert lib.sn_create_network(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.SN_EINVAL
    d = _desc()
    d.reset_scalar = float("inf")
    assert lib.sn_create_network(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.SN_EINVAL
    assert lib.sn_create_network(None, None, None, ctypes.byref(out)) == _lib.SN_EINVAL


def test_null_network_calls(lib):
    assert lib.sn_run(None, 5) == _lib.SN_EINVAL
    assert lib.sn_set_path(None, 0) == _lib.SN_EINVAL
    assert lib.sn_read_state(None, None, None) == _lib.SN_EINVAL
    assert lib.sn_load_dense_rows_i8(None, 0, 0, None, 6) == _lib.SN_EINVAL
    lib.sn_destroy_network(None)


def test_pack_unpack_roundtrip():
    import numpy as np
    from paper_2305_02510_amd.network import pack_bits, unpack_bits
    rng = np.random.default_rng(0)
    for n in (1, 31, 32, 33, 64, 65, 130):
        x = (rng.random((2, 3, n)) < 0.4).astype(np.uint8)
        w = pack_bits(x)
        assert w.shape == (2, 3, (n + 31) // 32)
        assert np.array_equal(unpack_bits(w, n), x)
        j = n - 1
        assert (w[..., j // 32] >> (j % 32) & 1 == x[..., j]).all()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no CPU fallback: without the built library the binding refuses to load
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        _lib.load()


def test_network_needs_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2305_02510_amd import Network
    with pytest.raises(RuntimeError, match="no GPU"):
        Network(10)


def test_package_never_uses_the_oracle():
    # the product path shares no code with the oracle and never imports it
    pkg = os.path.join(ROOT, "paper_2305_02510_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, flags=re.M), f
                assert "lif_oracle" not in text and "liboracle" not in text, f
