"""Benchmark: synaptic events per second of the LIF-with-delays simulation on
one MI355X, with the roofline fraction of the dominant kernel and the CPU
oracle timed beside it.

One benchmark step = one full simulation of the workload (state reset, then
all T time steps of delivery + neuron update) on inputs already resident in
device memory.  Workloads:

  large_sparse (default)  N = 10,000, directed Erdos-Renyi p = 0.01 (~1M
                          synapses), delays 1..16, T = 1000
  large_sparse_low        the same graph with inhibition-dominated weights
                          (firing rate ~0.2%), event-driven delivery
  dense_trials            N = 4096 dense weights, 64 trials, delay 1,
                          T = 1000, matrix cores
  uneven_batch            512 independent nets, N 50..5000, T = 500: one
                          batched persistent launch vs one run per net
  large_sparse_stdp       large_sparse with the plasticity rule on (window 8,
                          per-step path): simulation + weight updates
  paper_scale_dense       the paper's largest run: N = 100,000 all-to-all
                          dense delay-1 weights (int8 numerators, 10 GB in
                          HBM), one trial, T = 1000; each step reads only the
                          rows of the neurons that spiked
  bptt                    surrogate-gradient training step of a recurrent
                          layer: N = 2048, 256 inputs, 128 trials, T = 200
                          (forward + backward through time), FP32 matrix cores

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

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16 matrix cores, TFLOP/s
FP32_PEAK_TFLOPS = 157.3    # MI355X dense fp32 (matrix cores), TFLOP/s
INT8_PEAK_TOPS = 5000.0     # MI355X dense int8 matrix cores, TOP/s


def events_of(raster_btn: np.ndarray, out_degree: np.ndarray) -> int:
    """Synaptic events: every spike of neuron i is delivered over its out-degree synapses."""
    counts = raster_btn.sum(axis=(0, 1), dtype=np.int64)
    return int(counts @ out_degree)


def algorithmic_bytes_per_step(events: int, steps: int, n: int, trials: int) -> float:
    """Bytes a delivery + update time step must move at minimum: one 8-byte
    record (weight, source index and delay) per synaptic event, plus the
    neuron state read and written (V 4 + 4 bytes, refractory counter 1 + 1)
    per neuron and trial."""
    return 8.0 * events / steps + 10.0 * n * trials


LAST_TIMING = {}


def timed(fn, stream, warmup, steps):
    """Mean ms per call of fn over `steps` calls after `warmup` untimed ones,
    from HIP events on `stream` (the stream the library's kernels run on).
    An event between calls also gives each call's time; their median is kept
    in LAST_TIMING."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    each = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    LAST_TIMING["median_ms"] = float(np.median(each))
    LAST_TIMING["min_ms"] = float(np.min(each))
    return ev[0].elapsed_time(ev[steps]) / steps, wall


def host_cpu():
    """Cores this process may use and the CPU model of the host the oracle
    runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "model": model}


def median_time(fn, reps=3):
    """Median wall seconds of `reps` calls of fn, and the last call's result."""
    times, res = [], None
    for _ in range(reps):
        c0 = time.perf_counter()
        res = fn()
        times.append(time.perf_counter() - c0)
    return float(np.median(times)), res


def measured_traffic(summary: str, source: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary under
    profiles/, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    vals = dict(l.split(None, 1) for l in open(path) if l.strip() and not l.startswith("#"))
    cur = hashlib.sha256(open(os.path.join(ROOT, "paper_2305_02510_amd", "csrc", source), "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256", "").strip() != cur:
        return None
    return {"bytes_per_launch": int(float(vals["traffic_bytes_per_launch"])),
            "time_steps_per_launch": int(vals["time_steps_per_launch"]), "source": f"profiles/{summary}"}


# plasticity rule of the large_sparse_stdp workload (amplitudes k/64)
STDP_WINDOW = 8
STDP_LTP = [16 / 64, 8 / 64, 4 / 64, 2 / 64, 1 / 64, 1 / 64, 1 / 64, 1 / 64]
STDP_LTD = [12 / 64, 6 / 64, 3 / 64, 2 / 64, 1 / 64, 1 / 64, 1 / 64, 1 / 64]
STDP_CLIP = (-0.5, 1.0)


def bench_single(args, net, kind):
    """One net (possibly many trials): reset + run(T) per benchmark step.
    kind "stdp": plasticity on; the weights keep learning across the timed
    runs, and a last run from the loaded weights is checked against the
    oracle."""
    from paper_2305_02510_amd import Network
    T = net.steps
    t_setup = time.perf_counter()
    g = Network.from_workload(net)  # layout build (host) + uploads: setup, outside the timed region
    g.synchronize()
    setup_s = time.perf_counter() - t_setup
    tuned = None
    if kind == "stdp":
        g.set_stdp(STDP_WINDOW, STDP_LTP, STDP_LTD, *STDP_CLIP)  # runs on the per-step path
    elif args.path == "autotune":  # the library's autotuner picks path and slice count
        tuned = g.autotune(min(T, 128))
    else:
        g.set_path(args.path)

    def one_run():
        g.reset_state()
        g.run(T)

    ms, wall = timed(one_run, g.stream, args.warmup, args.steps)
    if kind == "stdp":  # the checked run starts from the loaded weights (setup, untimed)
        g.load_weights_delays(net.pre, net.post, net.weight, net.delay)
        one_run()
        weights = g.read_weights()
    raster = g.read_raster(0, T)
    V, ref = g.read_state()
    path = g.progress[1]
    g.close()
    ev = events_of(raster, net.out_degree())
    out = {"value": ev / (ms / 1e3), "ms_per_step": ms, "wall": wall, "events_per_run": ev,
           "mean_firing_rate": float(raster.mean()), "path": path, "autotuned": tuned, "setup_s": setup_s,
           "neuron_updates_per_s": net.n * net.trials * T / (ms / 1e3)}
    sec_per_tstep = ms / 1e3 / T
    if kind == "dense":
        # the contraction runs on int8 matrix cores when the weights allow it
        # (integer numerators over one power of two), else on bfloat16 ones
        i8 = path == "dense_persist_i8"
        flops = 2.0 * net.trials * net.n * net.n
        achieved = flops / sec_per_tstep / 1e12
        peak = INT8_PEAK_TOPS if i8 else BF16_PEAK_TFLOPS
        w_bytes = (1.0 if i8 else 2.0) * net.n * net.n
        out["dtype"] = "i8 x i8 -> i32" if i8 else "bf16 x bf16 -> f32"
        out["roofline"] = {
            "bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TOP/s" if i8 else "TFLOP/s",
            "frac": round(achieved / peak, 5), "traffic": None,
            "kernel": {"dense_persist_i8": "k_dense_persist<true>", "dense_persist": "k_dense_persist<false>"}.get(
                path, "k_dense_step"),
            "flops_per_time_step": flops, "us_per_time_step": round(sec_per_tstep * 1e6, 3),
            "weight_stream_GBps": round(w_bytes / sec_per_tstep / 1e9, 1),
            "weight_stream_frac_of_hbm": round(w_bytes / sec_per_tstep / 1e9 / HBM_PEAK_GBS, 4)}
    else:
        bytes_step = algorithmic_bytes_per_step(ev, T, net.n, net.trials)
        achieved = bytes_step / sec_per_tstep / 1e9
        # the per-step path stages the spike history through LDS in delay
        # phases (k_step_wide) once its 2*D words per 64-neuron group pass 64 KiB
        wide = 8 * net.max_delay * -(-net.n // 64) > 64 * 1024
        kernel = {"persist": "k_sim (multi-slice)", "small": "k_sim (one slice)",
                  "step": "k_step_wide (blocks of 4 steps)" if wide else "k_step", "push": "k_push"}.get(path, path)
        if kind == "stdp":
            kernel = "k_step + k_stdp (per step)"
        traffic = None
        if path == "persist" and net.name.startswith("large_sparse_n10000") and (tuned is None or tuned[1] == 0):
            # counters taken on the default slice plan
            traffic = measured_traffic("large_sparse_k_sim_persist_hbm_traffic.txt", "kernels.hip")
        for p_xl in ("0.01", "0.001"):
            if path == "step" and wide and net.name == f"large_sparse_xl_n100000_p{p_xl}":
                traffic = measured_traffic(f"large_sparse_xl_p{p_xl}_k_step_wide_hbm_traffic.txt", "wide.hip")
        out["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic["bytes_per_launch"] if traffic else None, "kernel": kernel,
            "bytes_per_time_step": round(bytes_step), "us_per_time_step": round(sec_per_tstep * 1e6, 3)}
        out["roofline"]["achieved_counts"] = ("algorithmic bytes: 8 B per synaptic event + 10 B of state per neuron "
                                              "and trial, per time step")
        if traffic:
            out["roofline"]["traffic_note"] = (f"HBM bytes per launch of {traffic['time_steps_per_launch']} time steps "
                                               f"(rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated; {traffic['source']})")
            hbm = traffic["bytes_per_launch"] / traffic["time_steps_per_launch"] / sec_per_tstep / 1e9
            out["roofline"]["hbm_measured_GBps"] = round(hbm, 2)
            out["roofline"]["hbm_measured_frac"] = round(hbm / HBM_PEAK_GBS, 5)
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        trials = list(range(min(net.trials, args.cpu_trials)))
        if kind == "stdp":
            def one():
                res = orc.stdp(net, STDP_WINDOW, STDP_LTP, STDP_LTD, *STDP_CLIP)
                res.spikes, res.V, res.ref = res.spikes[None], res.V[None], res.ref[None]
                return res
        elif kind == "dense":
            W64 = np.ascontiguousarray(net.dense_weight, np.float64)
            one = lambda: orc.run_dense(net, trials=trials, W=W64)
        else:
            one = lambda: orc.run_sparse(net, trials=trials, steps=cpu_steps)
        # a bounded sample: the first cpu_steps steps of the largest nets
        # (about 1.2e9 synapse-steps), every step otherwise
        cpu_steps = T if kind != "sparse" else int(min(T, max(10, 1.2e9 // max(1, net.nnz))))
        reps = args.cpu_reps
        if cpu_steps < T:
            c0 = time.perf_counter()
            res = one()
            first = time.perf_counter() - c0
            reps = 1 if first > 10 else args.cpu_reps
            csec, res = (first, res) if reps == 1 else median_time(one, reps)
        else:
            csec, res = median_time(one, reps)
        ev_cpu = events_of(res.spikes, net.out_degree())
        out["cpu_baseline"] = {
            "value": round(ev_cpu / csec, 1), "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(trials)} of {net.trials} trial(s), " + (f"all {T} steps" if cpu_steps == T else
                                                                     f"the first {cpu_steps} of {T} steps")
                      + f", N={net.n}, nnz={net.nnz}: median of {reps} single-threaded run(s), {csec:.2f} s",
            "host": host_cpu()}
        if cpu_steps == T:
            ok = (np.array_equal(raster[trials], res.spikes) and np.array_equal(V[trials].astype(np.float64), res.V)
                  and np.array_equal(ref[trials].astype(np.int32), res.ref)
                  and (kind != "stdp" or np.array_equal(weights.astype(np.float64), res.weight)))
        else:  # the oracle ran a prefix: the raster prefix is checked here, the rest below
            ok = np.array_equal(raster[trials][:, :cpu_steps], res.spikes)
        checked = trials
        if net.trials > 1:
            # all cores: one single-threaded oracle run per trial, every trial
            # (this is also the parity check of the whole run)
            workers = oracle.host_workers()
            rest = [b for b in range(net.trials) if b not in trials]
            run1 = (lambda b: orc.run_dense(net, trials=[b], W=W64)) if kind == "dense" else (
                lambda b: orc.run_sparse(net, trials=[b]))
            c0 = time.perf_counter()
            parts = oracle.fan_out(run1, range(net.trials), workers)
            asec = time.perf_counter() - c0
            ev_all = sum(events_of(p.spikes, net.out_degree()) for p in parts)
            for b, p in enumerate(parts):
                ok = ok and (np.array_equal(raster[b], p.spikes[0])
                             and np.array_equal(V[b].astype(np.float64), p.V[0])
                             and np.array_equal(ref[b].astype(np.int32), p.ref[0]))
            checked = trials + rest
            out["cpu_baseline"]["all_cores"] = {
                "value": round(ev_all / asec, 1), "unit": "synaptic events/s", "cores": workers,
                "sample": f"all {net.trials} trials, one single-threaded oracle run per trial on {workers} "
                          f"threads: {asec:.2f} s"}
        elif kind == "sparse":
            # all cores: the history-driven oracle on post ranges, driven by
            # the GPU raster; every range checked = the whole run, by induction
            # over t (each step's spikes depend only on earlier steps)
            workers = oracle.host_workers()
            ranges = oracle.post_ranges(net, 4 * workers)

            def rng_ok(r):
                j0, j1, idx = r
                p = orc.run_sparse_driven(net, raster, syn_index=idx)
                return (np.array_equal(raster[:, :, j0:j1], p.spikes[:, :, j0:j1])
                        and np.array_equal(V[:, j0:j1].astype(np.float64), p.V[:, j0:j1])
                        and np.array_equal(ref[:, j0:j1].astype(np.int32), p.ref[:, j0:j1]))
            c0 = time.perf_counter()
            oks = oracle.fan_out(rng_ok, ranges, workers)
            asec = time.perf_counter() - c0
            ok = ok and all(oks)
            out["cpu_baseline"]["all_cores"] = {
                "value": round(ev / asec, 1), "unit": "synaptic events/s", "cores": workers,
                "sample": f"all {T} steps, the history-driven oracle on {len(ranges)} post ranges (driven by the "
                          f"GPU raster) on {workers} threads: {asec:.2f} s"}
            out["parity_by_post_ranges"] = (f"every post range of the whole run recomputed from the GPU raster "
                                            f"({len(ranges)} ranges)")
        else:
            out["cpu_baseline"]["all_cores"] = None
            out["cpu_baseline"]["all_cores_note"] = "one trial with plasticity: no independent runs to spread"
        out["parity_bit_exact"] = bool(ok)
        out["parity_sample"] = (f"all {net.trials} trials" if len(checked) == net.trials
                                else f"trials {sorted(checked)}")
        if "parity_by_post_ranges" in out:
            out["parity_sample"] += "; " + out.pop("parity_by_post_ranges")
    return out


def bench_rows(args):
    """The paper's largest run (N = 100,000 all-to-all, one trial, T = 1000)
    on the dense-rows path: reset + run(T) per benchmark step.  The CPU leg
    runs the oracle on sampled neurons, each driven by the GPU raster, and
    checks their spikes and final state."""
    from paper_2305_02510_amd import Network
    from paper_2305_02510_amd import workloads as wl
    net = wl.paper_scale_dense()
    T, N = net.steps, net.n
    posts = np.sort(np.random.default_rng(5).choice(N, args.cpu_posts, replace=False)).astype(np.int32)
    t_setup = time.perf_counter()
    g, cols = Network.from_rows_workload(net, posts=posts, workers=16)  # draw + upload 10 GB: setup
    g.synchronize()
    setup_s = time.perf_counter() - t_setup
    tuned = None
    if args.path == "autotune":
        tuned = g.autotune(min(T, 128))
    else:
        g.set_path(args.path)

    def one_run():
        g.reset_state()
        g.run(T)

    ms, wall = timed(one_run, g.stream, args.warmup, args.steps)
    raster = g.read_raster(0, T)
    V, ref = g.read_state()
    path = g.progress[1]
    out_degree = g.out_degree
    g.close()
    ev = events_of(raster, out_degree)
    sec_per_tstep = ms / 1e3 / T
    # algorithmic bytes: the int8 row of every neuron that spiked the step
    # before (N bytes), plus the neuron state read and written
    row_bytes = float(raster[0, :-1].sum()) * N / T
    bytes_step = row_bytes + 10.0 * N
    achieved = bytes_step / sec_per_tstep / 1e9
    out = {"value": ev / (ms / 1e3), "ms_per_step": ms, "wall": wall, "events_per_run": ev,
           "mean_firing_rate": float(raster.mean()), "path": path, "autotuned": tuned, "setup_s": setup_s,
           "neuron_updates_per_s": N * T / (ms / 1e3), "dtype": "i8 -> i32",
           "config": {"workload": f"{net.name}: N={N} all-to-all dense delay-1 weights (int8 k/64, "
                                  f"{int(out_degree.sum())} non-zero), trials=1, T={T}",
                      "time_steps_per_run": T, "trials": 1}}
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_dense_rows",
        "bytes_per_time_step": round(bytes_step), "us_per_time_step": round(sec_per_tstep * 1e6, 3),
        "spiking_rows_per_time_step": round(float(raster[0, :-1].sum()) / T, 1)}
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        c0 = time.perf_counter()
        res = orc.run_columns(net, posts, cols.astype(np.float64) / 64.0, raster)
        csec = time.perf_counter() - c0
        counts = raster.sum(axis=(0, 1), dtype=np.int64)
        ev_cpu = int(((cols != 0) @ counts).sum())
        out["cpu_baseline"] = {
            "value": round(ev_cpu / csec, 1), "unit": "synaptic events/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{len(posts)} of {N} neurons, each over all {T} steps driven by the GPU raster "
                      f"(the oracle's column-wise dense update): {csec:.2f} s single-threaded"}
        # sampled columns driven by the GPU raster: not whole-network parity
        # (every column of a 50,000-neuron net is checked by the GPU tests)
        out["parity_bit_exact"] = None
        out["parity_sampled_columns_exact"] = bool(
            np.array_equal(raster[:, :, posts], res.spikes) and np.array_equal(V[:, posts].astype(np.float64), res.V)
            and np.array_equal(ref[:, posts].astype(np.int32), res.ref))
        out["parity_sample"] = f"{len(posts)} sampled neurons, all steps, each driven by the GPU raster"
    return out


def bench_batch(args, steps=None, warmup=None):
    """512 uneven nets: one batched persistent launch per benchmark step,
    compared with one run per net (each net on its own best single-net path,
    one after another on the same stream).  The CPU leg runs the oracle on
    every net (all cores: one single-threaded run per net), which is also the
    per-net parity check."""
    from paper_2305_02510_amd import Batch, Network
    from paper_2305_02510_amd import workloads as wl
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    nets = wl.uneven_batch(4)
    T = nets[0].steps
    t_setup = time.perf_counter()
    gs = [Network.from_workload(net) for net in nets]
    batch = Batch(gs)
    batch.synchronize()
    setup_s = time.perf_counter() - t_setup
    stream = gs[0].stream
    tuned = batch.autotune(min(T, 100)) if args.path == "autotune" else None  # the schedule autotuner

    def batched():
        for g in gs:
            g.reset_state()
        batch.run(T)

    def plain():
        for g in gs:
            g.reset_state()
            g.run(T)

    ms_b, wall = timed(batched, stream, warmup, steps)
    med_b = LAST_TIMING["median_ms"]
    rasters = [g.read_raster(0, T) for g in gs]
    states = [g.read_state() for g in gs]
    ms_p = None if args.no_plain else timed(plain, stream, 1, max(1, steps // 2))[0]
    ev_each = [events_of(r, net.out_degree()) for r, net in zip(rasters, nets)]
    ev = sum(ev_each)
    nnz = sum(net.nnz for net in nets)
    neurons = sum(net.n for net in nets)
    sec_per_tstep = ms_b / 1e3 / T
    bytes_step = 8.0 * ev / T + 10.0 * neurons
    achieved = bytes_step / sec_per_tstep / 1e9
    out = {"value": ev / (ms_b / 1e3), "ms_per_step": ms_b, "ms_per_step_median": med_b, "wall": wall,
           "events_per_run": ev, "mean_firing_rate": float(np.mean([r.mean() for r in rasters])), "path": "batch",
           "neuron_updates_per_s": neurons * T / (ms_b / 1e3), "setup_s": setup_s,
           "plain_ms_per_run": round(ms_p, 4) if ms_p else None,
           "batched_speedup_vs_plain": round(ms_p / ms_b, 3) if ms_p else None,
           "nets": len(nets), "total_neurons": neurons, "total_synapses": nnz,
           "schedule": {"target_mult": tuned[0], "team_share": tuned[1]} if tuned else None}
    traffic = measured_traffic("uneven_batch_k_batch_hbm_traffic.txt", "kernels.hip")
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "k_batch", "bytes_per_time_step": round(bytes_step), "us_per_time_step": round(sec_per_tstep * 1e6, 3),
        "achieved_counts": "algorithmic bytes: 8 B per synaptic event + 10 B of state per neuron, per time step"}
    if traffic:
        out["roofline"]["traffic_note"] = (f"HBM bytes per launch of {traffic['time_steps_per_launch']} time steps "
                                           f"(rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated; {traffic['source']})")
        out["roofline"]["hbm_measured_GBps"] = round(traffic["bytes_per_launch"] / (ms_b / 1e3) / 1e9, 1)
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        order = list(np.argsort([net.nnz for net in nets]))
        picks = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})

        def sample():
            return [orc.run_sparse(nets[i]) for i in picks]

        csec, _ = median_time(sample, args.cpu_reps)
        ev_sample = sum(ev_each[i] for i in picks)  # identical to the oracle's when parity holds
        workers = oracle.host_workers()
        longest_first = sorted(range(len(nets)), key=lambda i: -nets[i].nnz)
        c0 = time.perf_counter()
        res = dict(zip(longest_first, oracle.fan_out(lambda i: orc.run_sparse(nets[i]), longest_first, workers)))
        asec = time.perf_counter() - c0
        bad = [i for i in range(len(nets)) if not (
            np.array_equal(rasters[i], res[i].spikes) and np.array_equal(states[i][0].astype(np.float64), res[i].V)
            and np.array_equal(states[i][1].astype(np.int32), res[i].ref))]
        ev_cpu = sum(events_of(res[i].spikes, nets[i].out_degree()) for i in range(len(nets)))
        out["cpu_baseline"] = {
            "value": round(ev_sample / csec, 1), "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"nets {picks} (smallest, median and largest by synapses), all {T} steps: median of "
                      f"{args.cpu_reps} single-threaded runs, {csec:.2f} s",
            "host": host_cpu(),
            "all_cores": {"value": round(ev_cpu / asec, 1), "unit": "synaptic events/s", "cores": workers,
                          "sample": f"all {len(nets)} nets, one single-threaded oracle run per net on {workers} "
                                    f"threads: {asec:.2f} s"}}
        out["parity_bit_exact"] = not bad
        out["parity_sample"] = f"all {len(nets)} nets" + (f"; differing: {bad[:10]}" if bad else "")
    batch.close()
    for g in gs:
        g.close()
    return out


def bench_bptt(args):
    """One training step (forward with checkpoints + backward through time)
    of the recurrent LIF layer per benchmark step."""
    import torch
    from paper_2305_02510_amd import workloads as wl
    from paper_2305_02510_amd.bptt import spike_counts
    prob = wl.bptt_problem(5)
    T, B, Nin = prob.x.shape
    N = prob.W_rec.shape[0]
    Wr = torch.tensor(prob.W_rec, device="cuda", requires_grad=True)
    Wi = torch.tensor(prob.W_in, device="cuda", requires_grad=True)
    x = torch.tensor(prob.x, dtype=torch.float32, device="cuda")
    tgt = torch.tensor(prob.target, device="cuda")
    out_counts = {}

    def step():
        Wr.grad = None
        Wi.grad = None
        counts = spike_counts(Wr, Wi, x, prob.theta, prob.leak, prob.reset, prob.slope, prob.checkpoint)
        loss = ((counts / T - tgt) ** 2).mean()
        loss.backward()
        out_counts["c"] = counts

    stream = torch.cuda.current_stream()
    ms, wall = timed(step, stream, args.warmup, args.steps)
    counts = out_counts["c"].detach().cpu().numpy()
    # flops per training step by the unit they run on.  bfloat16 matrix cores:
    # the spike-operand products, each over the three exact bfloat16 pieces of
    # its other operand (forward spike term s(t-1) W_rec, its recomputation in
    # the backward pass, the W_rec gradient sum s(t-1)^T g): 3 x 3 x 2 T B N^2.
    # FP32 matrix cores: the input term x W_in, the backward term g W_rec^T
    # and the W_in gradient: 2 T B (2 Nin N + N^2).
    sec = ms / 1e3
    bf16_flops = 18.0 * T * B * N * N
    fp32_flops = 2.0 * T * B * (2 * Nin * N + N * N)
    algo_flops = 2.0 * T * B * N * (2 * (N + Nin) + N)  # the products of the method, counted once
    out = {"value": 1e3 / ms, "ms_per_step": ms, "wall": wall, "path": "bptt",
           "mean_firing_rate": float(counts.mean() / T),
           "neuron_updates_per_s": B * N * T / (ms / 1e3), "config": {
               "workload": f"bptt: recurrent N={N}, inputs={Nin}, trials={B}, T={T}, checkpoint every "
                           f"{prob.checkpoint} steps, dense delay-1 weights", "trials": B, "time_steps_per_run": T}}
    out["roofline"] = {"bound": "mfma", "achieved": round(bf16_flops / sec / 1e12, 3), "peak": BF16_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(bf16_flops / sec / 1e12 / BF16_PEAK_TFLOPS, 5),
                       "traffic": None,
                       "kernel": "k_gemm_split (spike-operand products on bfloat16 matrix cores, three exact pieces)",
                       "flops_per_step": bf16_flops,
                       "note": "bfloat16 flops executed per training step over the whole step's time: a lower bound "
                               "of the bfloat16 units' use (the FP32 products and epilogues share the step)"}
    out["roofline_fp32"] = {"bound": "mfma", "achieved": round(fp32_flops / sec / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": round(fp32_flops / sec / 1e12 / FP32_PEAK_TFLOPS, 5),
                            "kernel": "k_bptt_xw + k_bptt_part + k_bptt_wgrad (FP32 matrix cores)",
                            "flops_per_step": fp32_flops,
                            "note": "FP32 flops per training step over the whole step's time (lower bound)"}
    out["algorithmic_TFLOPs"] = round(algo_flops / sec / 1e12, 3)
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        # gradient of the last timed training step, all 128 trials
        gWr = Wr.grad.double().cpu().numpy()
        gWi = Wi.grad.double().cpu().numpy()
        one = lambda: orc.bptt(prob.W_rec, prob.W_in, prob.x[:, [0]], prob.target, prob.theta, prob.leak,
                               prob.reset, prob.slope)
        csec, _ = median_time(one, args.cpu_reps)
        # all cores: the batch gradient is the trial-count-weighted mean of the
        # gradients of trial subsets (the loss is a mean over trials)
        workers = oracle.host_workers()
        chunks = [list(range(i, min(B, i + 8))) for i in range(0, B, 8)]
        c0 = time.perf_counter()
        parts = oracle.fan_out(lambda tr: orc.bptt(prob.W_rec, prob.W_in, prob.x[:, tr], prob.target, prob.theta,
                                                   prob.leak, prob.reset, prob.slope), chunks, workers)
        asec = time.perf_counter() - c0
        dWr = sum(len(tr) / B * p.dW_rec for tr, p in zip(chunks, parts))
        dWi = sum(len(tr) / B * p.dW_in for tr, p in zip(chunks, parts))
        ref_counts = np.concatenate([p.counts for p in parts])
        out["cpu_baseline"] = {
            "value": round(1 / B / csec, 6), "unit": "training steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of {B} trials (a step's cost is linear in trials), all {T} steps: median of "
                      f"{args.cpu_reps} single-threaded runs, {csec:.2f} s",
            "host": host_cpu(),
            "all_cores": {"value": round(1 / asec, 6), "unit": "training steps/s", "cores": workers,
                          "sample": f"all {B} trials in {len(chunks)} single-threaded oracle runs of 8 trials on "
                                    f"{workers} threads: {asec:.2f} s"}}
        out["parity_bit_exact"] = None
        out["parity_counts_exact"] = bool(np.array_equal(counts, ref_counts))
        out["parity_grad_rel_err"] = float(np.linalg.norm(gWr - dWr) / np.linalg.norm(dWr))
        out["parity_grad_in_rel_err"] = float(np.linalg.norm(gWi - dWi) / np.linalg.norm(dWi))
        out["parity_sample"] = (f"the benchmarked step itself, all {B} trials: spike counts, and dW_rec / dW_in "
                                f"relative Frobenius error against the FP64 oracle (tolerance 1e-4)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_sparse",
                    choices=["large_sparse", "single_lif", "large_sparse_low", "dense_trials", "uneven_batch", "bptt",
                             "large_sparse_stdp", "paper_scale_dense", "large_sparse_xl_p0.001",
                             "large_sparse_xl_p0.01"])
    ap.add_argument("--path", default="autotune",
                    help="autotune (sn_autotune picks), auto (built-in heuristic) or a path name")
    ap.add_argument("--cpu-trials", type=int, default=2)
    ap.add_argument("--cpu-posts", type=int, default=16,
                    help="paper_scale_dense: neurons the oracle recomputes for the CPU leg and the parity check")
    ap.add_argument("--cpu-reps", type=int, default=3, help="single-threaded oracle runs; the median is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="uneven_batch: leave out the plain leg (one run per net), e.g. under a counter profiler, "
                         "which does not support the per-step paths' captured graphs")
    ap.add_argument("--no-batch", action="store_true",
                    help="large_sparse: leave out the uneven-batch (batched vs plain) leg of the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 256 MiB (read 256 MiB, write 256 MiB) and exit; "
                         "profiled with the same counters it scales FETCH_SIZE / WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: sharding the simulation across GPUs "
                                   "(post-neuron ranges with a per-step spike all-gather) is designed, not built"}))
        sys.exit(2)

    import torch
    from paper_2305_02510_amd import workloads as wl
    torch.cuda.set_device(0)

    if args.workload == "bptt":
        r = bench_bptt(args)
        out = {
            "metric": "training steps/sec", "value": round(r["value"], 4), "unit": "training steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded dense recurrent weights and Bernoulli input spikes)",
            "config": r["config"], "neuron_updates_per_s": round(r["neuron_updates_per_s"], 1),
            "mean_firing_rate": round(r["mean_firing_rate"], 5), "roofline": r["roofline"],
            "roofline_fp32": r.get("roofline_fp32"), "algorithmic_TFLOPs": r.get("algorithmic_TFLOPs"),
            "cpu_baseline": r.get("cpu_baseline"), "parity_counts_exact": r.get("parity_counts_exact"),
            "parity_grad_rel_err": r.get("parity_grad_rel_err"),
            "parity_grad_in_rel_err": r.get("parity_grad_in_rel_err"), "parity_sample": r.get("parity_sample"),
            "wall_s_timed": round(r["wall"], 4)}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "uneven_batch":
        r = bench_batch(args)
        desc = (f"uneven_batch: {r['nets']} independent nets, N log-uniform 50..5000 (total {r['total_neurons']}), "
                f"p 0.005..0.2 (total {r['total_synapses']} synapses), D 1..16, T=500")
        cfg = {"workload": desc, "nets": r["nets"], "time_steps_per_run": 500}
    elif args.workload == "paper_scale_dense":
        r = bench_rows(args)
        cfg = r["config"]
    else:
        net = wl.by_name("large_sparse" if args.workload == "large_sparse_stdp" else args.workload)
        kind = {"dense_trials": "dense", "large_sparse_stdp": "stdp"}.get(args.workload, "sparse")
        r = bench_single(args, net, kind)
        cfg = {"workload": f"{net.name}: N={net.n}, nnz={net.nnz}, D={net.max_delay}, T={net.steps}, "
                           f"trials={net.trials}" + (", STDP window 8" if kind == "stdp" else ""),
               "time_steps_per_run": net.steps, "trials": net.trials}
    cfg["path"] = r["path"]
    if r.get("autotuned"):
        cfg["autotuned"] = {"path": r["autotuned"][0], "slices": r["autotuned"][1]}
    out = {
        "metric": "synaptic events/sec", "value": round(r["value"], 1), "unit": "synaptic events/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": r.get("dtype", "f32"),
        "data": "synthetic (seeded Erdos-Renyi / dense nets and Bernoulli external spikes)",
        "config": cfg,
        "neuron_updates_per_s": round(r["neuron_updates_per_s"], 1),
        "events_per_run": r["events_per_run"], "mean_firing_rate": round(r["mean_firing_rate"], 5),
        "roofline": r["roofline"], "cpu_baseline": r.get("cpu_baseline"),
        "parity_bit_exact": r.get("parity_bit_exact"), "parity_sample": r.get("parity_sample"),
        "wall_s_timed": round(r["wall"], 4),
    }
    if "parity_sampled_columns_exact" in r:
        out["parity_sampled_columns_exact"] = r["parity_sampled_columns_exact"]
    if "setup_s" in r:  # network creation, layout build and upload, timed apart from the steps
        out["setup_s"] = round(r["setup_s"], 4)
    for k in ("plain_ms_per_run", "batched_speedup_vs_plain", "ms_per_step_median"):
        if k in r:
            out[k] = r[k]
    if r.get("schedule"):
        out["config"]["schedule_autotuned"] = r["schedule"]
    if "ms_per_step_median" not in out:
        out["ms_per_step_median"] = round(LAST_TIMING.get("median_ms", float("nan")), 4)
    if args.workload == "large_sparse" and not args.no_batch:
        # the metric's other half: many uneven nets in one batched launch
        # against one plain run per net, on the same GPU in the same job
        rb = bench_batch(args, steps=max(2, min(args.steps, 5)), warmup=1)
        out["batched_speedup_vs_plain"] = rb["batched_speedup_vs_plain"]
        out["uneven_batch"] = {
            "workload": (f"uneven_batch: {rb['nets']} independent nets, N log-uniform 50..5000 (total "
                         f"{rb['total_neurons']}), p 0.005..0.2 (total {rb['total_synapses']} synapses), D 1..16, "
                         f"T=500"),
            "value": round(rb["value"], 1), "unit": "synaptic events/s",
            "batched_ms_per_run": round(rb["ms_per_step"], 4),
            "batched_ms_per_run_median": round(rb["ms_per_step_median"], 4),
            "plain_ms_per_run": rb["plain_ms_per_run"],
            "batched_speedup_vs_plain": rb["batched_speedup_vs_plain"],
            "neuron_updates_per_s": round(rb["neuron_updates_per_s"], 1),
            "events_per_run": rb["events_per_run"], "roofline": rb["roofline"],
            "cpu_baseline": rb.get("cpu_baseline"), "parity_bit_exact": rb.get("parity_bit_exact"),
            "parity_sample": rb.get("parity_sample"), "setup_s": round(rb["setup_s"], 3),
            "schedule_autotuned": rb.get("schedule")}
    print(json.dumps(out), flush=True)


def release_device():
    """Every network and batch is closed by the legs above; drain the device
    and hand torch's cached blocks back before the interpreter exits, so no
    device memory or stream the library used outlives the program."""
    import gc
    import torch
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
    release_device()
