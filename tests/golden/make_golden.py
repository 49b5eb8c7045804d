"""Writes golden/single_lif_digest.txt from the CPU oracle (only the oracle and
the seeded generator are used)."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2305_02510_amd import workloads as wl  # noqa: E402

res = oracle.Oracle().run_sparse(wl.single_lif(1))
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_lif_digest.txt")
with open(out, "w") as f:
    f.write("# oracle on workloads.single_lif(seed=1): N=110, T=100; written by make_golden.py\n")
    f.write(f"spikes_sha256 {hashlib.sha256(res.spikes.tobytes()).hexdigest()}\n")
    f.write(f"V_sha256 {hashlib.sha256(res.V.astype('<f8').tobytes()).hexdigest()}\n")
    f.write(f"spike_count {int(res.spikes.sum())}\n")
print(open(out).read())
