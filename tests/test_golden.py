"""Oracle against hand-derived and stored values (tests/golden/)."""
import hashlib
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_pins import tiny_net  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_constant_drive_worked_example(oracle):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "constant_drive.txt")) if l.strip() and l[0] != "#"]
    assert rows
    for r in rows:
        theta, lam, a, R = float(r[0]), float(r[1]), float(r[2]), int(r[3])
        expect = [int(x) for x in r[4:]]
        net = tiny_net(1, steps=40, theta=theta, leak=lam, refractory=R, amplitude=a,
                       ext_events=[(0, t, 0) for t in range(40)])
        got = list(np.nonzero(oracle.run_sparse(net).spikes[0, :, 0])[0])
        assert got == expect, (r, got)


def test_single_lif_digest(oracle):
    """Regression digest of the oracle on the small seeded net, written by
    golden/make_golden.py (which calls only the oracle and the generator)."""
    from paper_2305_02510_amd import workloads as wl
    want = dict(l.split() for l in open(os.path.join(GOLDEN, "single_lif_digest.txt")) if l[0] != "#")
    res = oracle.run_sparse(wl.single_lif(1))
    assert res.exact
    assert hashlib.sha256(res.spikes.tobytes()).hexdigest() == want["spikes_sha256"]
    assert hashlib.sha256(res.V.astype("<f8").tobytes()).hexdigest() == want["V_sha256"]
    assert int(res.spikes.sum()) == int(want["spike_count"])
