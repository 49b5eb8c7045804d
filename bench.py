"""Benchmark: synaptic events per second of the LIF-with-delays simulation on
one MI355X, with the HBM roofline fraction of the dominant kernel and the CPU
oracle timed beside it.

One benchmark step = one full simulation of the workload (state reset, then
all T time steps of delivery + neuron update) on inputs already resident in
device memory.  The default workload is the large sparse net: N = 10,000
neurons, directed Erdos-Renyi p = 0.01 (~1M synapses), delays 1..16,
T = 1000 steps.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def events_of(raster_btn: np.ndarray, out_degree: np.ndarray) -> int:
    """Synaptic events: every spike of neuron i is delivered over its out-degree synapses."""
    counts = raster_btn.sum(axis=(0, 1), dtype=np.int64)
    return int(counts @ out_degree)


def algorithmic_bytes_per_step(events: int, steps: int, n: int, trials: int) -> float:
    """Bytes a delivery + update step must move at minimum: one 8-byte record
    (weight, source index and delay) per synaptic event, plus the neuron
    state read and written (V 4+4 bytes, refractory counter 1+1) per neuron."""
    return 8.0 * events / steps + 10.0 * n * trials


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_sparse",
                    choices=["large_sparse", "single_lif", "large_sparse_low"])
    ap.add_argument("--path", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is "
                          "described in DESIGN.md but not built"}))
        sys.exit(2)

    import torch
    from paper_2305_02510_amd import Network
    from paper_2305_02510_amd import workloads as wl

    torch.cuda.set_device(0)
    net = wl.by_name(args.workload)
    T = net.steps
    g = Network.from_workload(net)
    g.set_path(args.path)
    stream = g.stream

    def one_run():
        g.reset_state()
        g.run(T)

    for _ in range(args.warmup):
        one_run()
    g.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        one_run()
    stop.record(stream)
    g.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(stop)
    ms_per_step = gpu_ms / args.steps

    raster = g.read_raster(0, T)
    V, ref = g.read_state()
    path = g.progress[1]
    g.close()
    outdeg = net.out_degree()
    ev = events_of(raster, outdeg)
    value = ev / (ms_per_step / 1e3)
    rate = float(raster.mean())

    # roofline of the dominant kernel: algorithmic bytes of one time step over
    # the average time of one time step inside the timed region
    bytes_step = algorithmic_bytes_per_step(ev, T, net.n, net.trials)
    sec_per_tstep = ms_per_step / 1e3 / T
    achieved = bytes_step / sec_per_tstep / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": {"step": "k_step", "small": "k_small"}.get(path, path),
                "bytes_per_time_step": round(bytes_step), "us_per_time_step": round(sec_per_tstep * 1e6, 3)}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        c0 = time.perf_counter()
        res = orc.run_sparse(net)
        csec = time.perf_counter() - c0
        cpu = {"value": round(ev / csec, 1), "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
               "sample": f"one full run of the workload ({T} steps, N={net.n}, nnz={net.nnz}), "
                         f"{csec:.2f} s single-threaded"}
        parity = bool(np.array_equal(raster, res.spikes) and np.array_equal(V.astype(np.float64), res.V)
                      and np.array_equal(ref.astype(np.int32), res.ref))

    out = {
        "metric": "synaptic events/sec", "value": round(value, 1), "unit": "synaptic events/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Erdos-Renyi net and Bernoulli external spikes)",
        "config": {"workload": f"{net.name}: N={net.n}, nnz={net.nnz}, D={net.max_delay}, T={T}, "
                               f"trials={net.trials}", "path": path, "time_steps_per_run": T},
        "neuron_updates_per_s": round(net.n * net.trials * T / (ms_per_step / 1e3), 1),
        "events_per_run": ev, "mean_firing_rate": round(rate, 5),
        "roofline": roofline, "cpu_baseline": cpu, "parity_bit_exact": parity,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
