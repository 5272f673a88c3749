"""Benchmark: vehicle-steps per second of the LPSim vehicle update on one MI355X.

Workload (the paper's single-GPU regional case at its published size, on
synthetic stand-ins for the SF Bay network and SFCTA demand): planar road
graph of 225,150 nodes and 550,000 directed edges, 2,820,000 routed trips over
a two-peak 3 h morning profile, dt = 0.5 s, horizon 28,800 steps.

A "step" is one simulation time step of every vehicle (move, resolve, lane
change, commit).  value = vehicle-steps / s over the timed steps (a
vehicle-step is one vehicle active at the start of a step), inputs resident in
device memory.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

With --steps K the timed window is K steps from the peak of load: the step at
which the most vehicles are on the road (found by an untimed pass over the
horizon), reached untimed and restored before each of the timed runs.
Without --steps the whole horizon from step 0 is timed.  The roofline entry
prices the dominant kernel's algorithmic bytes over the same window against
the MI355X HBM peak; `cpu_baseline` times the plain CPU oracle (one core and
all cores) on a bounded prefix of the same workload, with the GPU timed on
that same prefix beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the move launch per active vehicle-step, besides what
# the device counts into scan_bytes (lane-map cells scanned, one byte each;
# the next edge's entry window near the stop line; a crossing vehicle's trip
# id, claim word and request, 20; the departure requests' origin-lane list,
# lane record, head, trip id and entry-window reads, which run in the same
# launch).  The fixed part is what the method must move per vehicle-step, not
# what this kernel happens to read:
#   state read: x, v, edge, lane, status, route index (18)
#   state write: x, v (8)
# The kernel actually reads 28 bytes (meta, x, v and 16 bytes of edge data
# cached in the slot, in place of the edge id and route index) and writes 12
# (x, v, meta); the counted HBM traffic shows what it moves.
MOVE_FIXED_BYTES = 18 + 8

# HBM traffic of one k_move launch, from two rocprofv3 --pmc runs of the
# benchmark command itself (FETCH_SIZE, WRITE_SIZE: KiB per dispatch, mean
# over the dispatches of the timed window), each scaled by what the same
# counter reads for a plain device copy of known size.  A figure is reported
# only for the workload and window it was counted on, and only while the
# kernel source hashes to the value it was counted with; otherwise null.
MOVE_TRAFFIC = {
    # profiles/k_move_regional_peak_counters.md
    ("regional-225k-2.82M", 19136, 20): {
        "fetch_kib": 43035.53, "fetch_scale": 2.0, "write_kib": 24110.31, "write_scale": 1.0,
        "kernels_sha256": "9ed09b628f65469f4638b9ea73974b0949f5934106e95f402f81d8475339b5c3"},
}


def move_traffic_bytes(workload, start, steps):
    import hashlib

    t = MOVE_TRAFFIC.get((workload, start, steps))
    if t is None:
        return None
    src = os.path.join(ROOT, "paper_2406_08496_amd", "csrc", "lpsim_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if t["kernels_sha256"] != sha:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def summarize_profile(path, last):
    """Summary of a rocprofv3 CSV file of this benchmark's run: for each
    kernel, the mean over all its dispatches and over its LAST `last`
    dispatches, which are the roofline pass (the timed window's steps with
    the kernels launched one by one) when the run had no perceptron or CPU
    baseline leg.  A kernel trace (`*_kernel_trace.csv`) gives durations in
    microseconds; a counter file (`*_counter_collection.csv`) gives each
    counter's value per dispatch.  Prints a markdown table."""
    import csv
    from collections import defaultdict

    rows = defaultdict(list)
    with open(path, newline="") as f:
        rd = csv.DictReader(f)
        counters = "Counter_Name" in rd.fieldnames
        for r in rd:
            name = r["Kernel_Name"]
            key = (name, r["Counter_Name"]) if counters else (name, "duration_us")
            val = (float(r["Counter_Value"]) if counters
                   else (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            rows[key].append((int(r["Dispatch_Id"]), val))
    print(f"| kernel | quantity | dispatches | mean (all) | mean (last {last}) |")
    print("|---|---|---|---|---|")
    for (name, what), v in sorted(rows.items(), key=lambda kv: -sum(x for _, x in kv[1])):
        v.sort()
        tail = [x for _, x in v[-last:]]
        short = name.split("(")[0]
        print(f"| {short} | {what} | {len(v)} | {sum(x for _, x in v) / len(v):.2f} | "
              f"{sum(tail) / len(tail):.2f} |")


def make_workload(name):
    from paper_2406_08496_amd import synth

    if name.startswith("batch"):
        n = int(name.split(":")[1]) if ":" in name else 64
        return synth.batch_scenarios(n), 48
    if name == "regional":
        return synth.regional(), 48
    if name == "tiny":
        return synth.tiny_grid(), 12
    if name.startswith("regional:"):
        return synth.regional(float(name.split(":")[1])), 48
    if name.startswith("regional-demand:"):
        return synth.regional(1.0, demand=float(name.split(":")[1])), 48
    if name == "large":
        return synth.large(), 60
    if name.startswith("large:"):
        return synth.large(float(name.split(":")[1])), 60
    raise SystemExit(f"unknown workload {name}")


def host_cpu():
    """CPU model and hardware thread count of the host the oracle runs on."""
    import os
    import platform

    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "hardware_threads": os.cpu_count()}


def cpu_baseline(inst, n_bins, budget_s, plan=None):
    """The oracle as it is, on the host cores: the single-threaded build from
    step 0 until `budget_s` runs out (whole 100-step blocks), then the
    all-cores build (OpenMP, same results) over the same steps.  Returns the
    entry and the number of steps of the sample."""
    import oracle

    legs = {}
    steps = None
    for parallel in (False, True):
        o = oracle.OracleSim(parallel=parallel, n_bins=n_bins).load(inst)
        if plan is not None:
            o.set_signals(plan)
        t0 = time.perf_counter()
        done = 0
        while (done < steps) if steps is not None else (time.perf_counter() - t0 < budget_s
                                                         and done < inst.n_steps):
            o.step(100)
            done += 100
        el = time.perf_counter() - t0
        steps = done
        c = o.counters()
        legs[parallel] = {"value": c["vehicle_steps"] / el, "cores": o.threads, "seconds": el,
                          "vehicle_steps": c["vehicle_steps"]}
        del o
    par, one = legs[True], legs[False]
    out = {"value": par["value"], "unit": "vehicle-steps/s", "cores": par["cores"], "kind": "oracle",
           "sample": f"steps 0..{steps} of the same workload ({par['vehicle_steps']} vehicle-steps); "
                     f"all-cores build {par['seconds']:.1f} s on {par['cores']} threads, "
                     f"single-threaded build {one['seconds']:.1f} s",
           "single_thread": {"value": one["value"], "cores": 1, "seconds": one["seconds"]},
           "host": host_cpu()}
    return out, steps


def find_peak(sim, horizon, every=64):
    """Step from the current state to the horizon and return the step (a
    multiple of `every`) at which the most vehicles were on the road, with
    that count and the counters at the horizon."""
    best, best_k, k = -1, 0, 0
    while k < horizon:
        n = min(every, horizon - k)
        sim.step(n)
        k += n
        a = sim.counters()["active"]
        if a > best:
            best, best_k = a, k
    return best_k, best, sim.counters()


def window_state(sim, n_trips):
    """What the road looks like at the start of the timed window."""
    v = sim.vehicles()
    act = v["status"] == 1
    n_act = int(act.sum())
    stopped = int((act & (v["v"] == 0)).sum())
    c = sim.counters()
    return {"active": n_act, "stopped_share": stopped / max(n_act, 1),
            "waiting": c["waiting"], "arrived_fraction": c["arrived"] / max(n_trips, 1)}


CNT_DELTA = ("vehicle_steps", "transfers", "departures", "arrived", "claims_lost", "lc_attempts",
             "lc_accepts", "scan_bytes")


def delta(c1, c0):
    return {k: c1[k] - c0[k] for k in CNT_DELTA}


def step_bytes(d, look_ahead):
    """Algorithmic bytes of whole steps from the counters of the steps: per
    vehicle-step the state read (18: x, v, edge, lane, status, route index),
    x and v written (8) and the map commit (2); what the move launch counts
    into scan_bytes (cells scanned, entry windows near a stop line, entry
    requests, departure requests); 16 per exit (statistics), 20 per
    departure; two look-ahead windows per lane-change attempt."""
    exits = d["transfers"] + d["arrived"]
    return (28 * d["vehicle_steps"] + d["scan_bytes"] + 16 * exits + 20 * d["departures"]
            + 2 * look_ahead * d["lc_attempts"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps; without it the whole horizon from step 0 is timed")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--window-start", default=None,
                    help="first timed step: 'peak' (the step with the most vehicles on the road, "
                         "the default with --steps) or a step number (default 0 without --steps)")
    ap.add_argument("--repeat", type=int, default=3,
                    help="timed runs of the same steps from the same state; the median is reported")
    ap.add_argument("--workload", default="regional")
    ap.add_argument("--block", type=int, default=512)
    ap.add_argument("--blocks", type=int, default=640)
    ap.add_argument("--graph-steps", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of the single-threaded oracle leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--assign", type=int, default=0,
                    help="also run N MSA iterations, plain vs surrogate-assisted")
    ap.add_argument("--assign-workload", default=None,
                    help="instance of the assignment comparison (default: the bench workload), "
                         "e.g. regional-demand:0.25 for the regional network at a quarter of the demand")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape first")
    ap.add_argument("--signals", action="store_true",
                    help="fixed-time two-phase signals at every node with 3+ approaches on both axes")
    ap.add_argument("--no-mlp", action="store_true", help="skip the surrogate perceptron leg")
    ap.add_argument("--mlp-only", action="store_true", help="only run the surrogate perceptron leg")
    ap.add_argument("--mlp-samples", type=int, default=2_200_000,
                    help="inference batch of the perceptron leg (550k edges x 4 one-hour windows)")
    ap.add_argument("--route-only", type=int, default=0, metavar="N",
                    help="only time the routing step of N MSA iterations on the regional network "
                         "(GPU trees toward its 500 destinations, new routes for the switched trips)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale the HBM traffic counters")
    ap.add_argument("--summarize-profile", default=None, metavar="CSV",
                    help="only summarise a rocprofv3 kernel-trace or counter CSV of a run of this "
                         "benchmark, over all dispatches and over the last --steps of each kernel")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.steps or 20)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the simulator runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2406_08496_amd.lpsim import Simulator

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 5}), flush=True)
        return
    if args.mlp_only:
        print(json.dumps({"surrogate_mlp": run_mlp(args.mlp_samples, 8192)}), flush=True)
        return
    if args.route_only:
        print(json.dumps({"routing": run_routing(args.route_only)}), flush=True)
        return
    t = time.perf_counter()
    inst, n_bins = make_workload(args.workload)
    batch = isinstance(inst, list)
    if batch:
        insts = inst
        name = f"batch-{len(insts)}-scenarios"
        n_nodes = sum(i.n_nodes for i in insts)
        n_edges = sum(i.n_edges for i in insts)
        n_trips = sum(i.n_trips for i in insts)
        n_route = sum(int(i.route_off[-1]) for i in insts)
        horizon = max(i.n_steps for i in insts)
    else:
        name, n_nodes, n_edges, n_trips = inst.name, inst.n_nodes, inst.n_edges, inst.n_trips
        n_route, horizon = int(inst.route_off[-1]), inst.n_steps
    plan = None
    if args.signals:
        from paper_2406_08496_amd import synth

        plan = (synth.concat_signal_plans([synth.signal_plan(i) for i in insts], insts) if batch
                else synth.signal_plan(inst))
        name += "+signals"
    log(f"workload {name}: {n_nodes} nodes, {n_edges} edges, {n_trips} trips, "
        f"{n_route} route entries; generated in {time.perf_counter() - t:.1f} s")

    t = time.perf_counter()
    sim = Simulator(n_bins=n_bins)
    sim.set_launch(args.block, args.blocks, args.graph_steps)
    if batch:
        sim.load_batch(insts)
    else:
        sim.load(inst)
    if plan is not None:
        sim.set_signals(plan)
        log(f"signals at {plan.n_signals} nodes")
    log(f"loaded in {time.perf_counter() - t:.1f} s")
    stream = torch.cuda.current_stream()
    snap0 = sim.save_state()

    # the timed window: K steps from step P
    full = args.steps is None
    K = horizon if full else args.steps
    ws = args.window_start if args.window_start is not None else ("0" if full else "peak")
    horizon_info = None
    if ws == "peak":
        t = time.perf_counter()
        peak_k, peak_active, ch = find_peak(sim, horizon)
        P = min(peak_k, max(horizon - K, 0))
        horizon_info = {"active_peak": peak_active, "active_peak_step": peak_k,
                        "arrived_fraction": ch["arrived"] / n_trips, "vehicle_steps": ch["vehicle_steps"]}
        log(f"most vehicles on the road: {peak_active} at step {peak_k} (found in "
            f"{time.perf_counter() - t:.1f} s); horizon: arrived {ch['arrived']}/{n_trips}")
        sim.restore_state(snap0)
    else:
        P = int(ws)
    if P:
        sim.step(P)
    snapP = sim.save_state() if P else snap0
    win = window_state(sim, n_trips)
    c_start = sim.counters()
    log(f"window: steps {P}..{P + K}; at its start {win['active']} vehicles on the road "
        f"({100 * win['stopped_share']:.1f}% standing), {win['waiting']} trips waiting")
    tuned = None
    if args.autotune:
        tuned = sim.autotune(n_steps=64)
        log(f"autotuned on the window state: block {tuned['block_size']}, blocks {tuned['blocks']}")
        tuned = {"block": tuned["block_size"], "blocks": tuned["blocks"],
                 "trial_us_per_step": {f"{b}x{g}": round(u, 2) for (b, g), u in tuned["us_per_step"].items()}}
    # warm-up steps (graph capture, caches), then rewind to the window start
    W = args.warmup
    if W:
        sim.step(W, stream=stream)
        torch.cuda.synchronize()
    sim.restore_state(snapP)
    # capture the graphs of a K-step call outside the timed region
    sim.prepare(K)

    runs = []
    for r in range(max(1, args.repeat)):
        if r:
            sim.restore_state(snapP)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        t0 = time.perf_counter()
        sim.step(K, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs.append((ev0.elapsed_time(ev1), wall))
        log(f"run {r}: {runs[-1][0]:.2f} ms")
    ms, wall = sorted(runs)[len(runs) // 2]
    c_end = sim.counters()
    dw = delta(c_end, c_start)
    vsteps = dw["vehicle_steps"]
    value = vsteps / (ms / 1e3)
    win["arrived_fraction_end"] = c_end["arrived"] / n_trips
    win["mean_active"] = vsteps / K
    log(f"timed {K} steps: {ms:.2f} ms (wall {wall * 1e3:.2f} ms), {vsteps} vehicle-steps, "
        f"arrived {c_end['arrived']}/{n_trips}, active {c_end['active']}, watchdog {c_end['watchdog']}")

    cfg = {"workload": name, "nodes": n_nodes, "edges": n_edges, "trips": n_trips, "dt": 0.5,
           "horizon_steps": horizon, "window_start_step": P, "window_steps": K,
           "block": tuned["block"] if tuned else args.block,
           "blocks": tuned["blocks"] if tuned else args.blocks, "graph_steps": args.graph_steps,
           "signalised_nodes": plan.n_signals if plan is not None else 0}
    out = {
        "metric": (f"vehicle-steps/sec, {len(insts)} batched scenarios" if batch else
                   f"vehicle-steps/sec at {n_trips / 1e6:.3g}M trips".replace("2.82M", "2.8M")),
        "value": value,
        "unit": "vehicle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded planar graph + gravity demand standing in for SF Bay / SFCTA)",
        "config": cfg,
        "window": win,
        "trips_per_s": (c_end["arrived"] - c_start["arrived"]) / (ms / 1e3),
        "vehicle_steps": vsteps,
        "window_counters": dw,
        "runs_ms": [round(x[0], 3) for x in runs],
    }
    if horizon_info is not None:
        out["horizon"] = horizon_info
    if tuned:
        out["autotune"] = tuned

    if not args.no_roofline:
        # the same K steps from the same state, kernels launched one by one
        # with their dispatch timestamps taken by HIP events on the work stream
        sim.restore_state(snapP)
        c0 = sim.counters()
        sim.set_timing(True)
        sim.step(K, stream=stream)
        torch.cuda.synchronize()
        times = sim.kernel_times()
        d2 = delta(sim.counters(), c0)
        sim.set_timing(False)
        dom = max(times, key=lambda k: times[k][0])
        alg_bytes = MOVE_FIXED_BYTES * d2["vehicle_steps"] + d2["scan_bytes"]
        mv_ms, mv_n = times["move"]
        achieved = alg_bytes / (mv_ms / 1e3) / 1e9
        traffic = move_traffic_bytes(name, P, K)
        out["roofline"] = {"bound": "hbm", "kernel": "k_move", "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": traffic,
                           "bytes_per_launch": alg_bytes / max(mv_n, 1),
                           "avg_launch_us": mv_ms * 1e3 / max(mv_n, 1)}
        sb = step_bytes(dw, sim.D)
        step_gbs = sb / (ms / 1e3) / 1e9
        out["step_roofline"] = {"bound": "hbm", "achieved": step_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": step_gbs / HBM_PEAK_GBS, "bytes_per_step": sb / K}
        out["kernel_ms"] = {k: {"total_ms": v[0], "launches": v[1],
                                "avg_us": (v[0] * 1e3 / v[1]) if v[1] else None}
                            for k, v in times.items()}
        out["dominant_kernel"] = dom
        log("kernel times:", json.dumps(out["kernel_ms"]))

    if not args.no_mlp:
        out["surrogate_mlp"] = run_mlp(args.mlp_samples, 8192)
        log("surrogate perceptron:", json.dumps(out["surrogate_mlp"]))
    if not args.no_cpu_baseline and not batch:
        cb, s_steps = cpu_baseline(inst, n_bins, args.cpu_budget, plan)
        # the GPU on exactly the oracle's sample, for the comparison
        sim.restore_state(snap0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(s_steps, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        g_ms = e0.elapsed_time(e1)
        g_vs = sim.counters()["vehicle_steps"]
        cb["gpu_same_sample"] = {"value": g_vs / (g_ms / 1e3), "ms": g_ms,
                                 "vs_all_cores": (g_vs / (g_ms / 1e3)) / cb["value"]}
        out["cpu_baseline"] = cb
        log("cpu baseline:", json.dumps(out["cpu_baseline"]))
    if args.assign and not batch:
        a_inst = inst if args.assign_workload is None else make_workload(args.assign_workload)[0]
        out["assignment"] = run_assignment(a_inst, args.assign)
        out["assignment"]["workload"] = a_inst.name
    print(json.dumps(out), flush=True)


# perceptron FLOPs per sample: forward over the four layers as computed (16
# outputs); backward = weight gradients of all four layers + data gradients of
# layers 2..4 (the input needs none)
MLP_DIMS = ((32, 256), (256, 256), (256, 256), (256, 16))
MLP_FWD_FLOP = sum(2 * i * o for i, o in MLP_DIMS)
MLP_BWD_FLOP = MLP_FWD_FLOP + sum(2 * i * o for i, o in MLP_DIMS[1:])
BF16_PEAK_TFLOPS = 2500.0


def run_mlp(n_fwd, n_train, reps=10):
    """Time the surrogate perceptron's MFMA kernels with HIP events on the
    stream they run on: the forward over an inference batch (every edge and
    one-hour window of the regional network), and the backward over a training
    batch and over the inference batch."""
    import torch
    from paper_2406_08496_amd.surrogate import EdgeMLP

    net = EdgeMLP(seed=0)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def entry(flop, ms):
        tf = flop / (ms / 1e3) / 1e12
        return {"ms": ms, "tflops": tf, "frac": tf / BF16_PEAK_TFLOPS}

    out = {"bound": "mfma", "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "dtype": "bf16 operands, f32 accumulation",
           "flop_per_sample": {"forward": MLP_FWD_FLOP, "backward": MLP_BWD_FLOP}}
    x = torch.randn((n_fwd, 32), generator=g, device="cuda").to(torch.bfloat16)
    out["forward"] = dict(entry(MLP_FWD_FLOP * n_fwd, timed(lambda: net.forward(x))), samples=n_fwd)
    for name, n in (("backward_train_batch", n_train), ("backward", n_fwd)):
        xb = x[:n].contiguous()
        tgt = torch.randn((n, 16), generator=g, device="cuda")
        y, hs = net.forward(xb, keep=True)
        dz = torch.empty((n, 16), dtype=torch.bfloat16, device="cuda")
        lib = net.lib
        import ctypes
        rc = lib.lpsim_mlp_loss_grad(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(tgt.data_ptr()), None, n,
                                     ctypes.c_float(1.0 / (n * 16)), ctypes.c_void_p(dz.data_ptr()), None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if rc:
            raise RuntimeError(f"mlp loss gradient failed: {rc}")
        out[name] = dict(entry(MLP_BWD_FLOP * n, timed(lambda: net.backward(xb, hs, dz))), samples=n)
        del y, hs, dz, tgt, xb
    return out


def run_routing(n_iter, seed=11):
    """The routing step of MSA iterations 1..n_iter on the regional network,
    on its own: edge costs are the free-flow times times a seeded log-normal
    congestion factor (a new draw each iteration), the switch moves 1/(n+1)
    of the trips, and each iteration's routes start from the last ones, as
    in the loop.  Host wall clock per iteration: the tree solve and writing
    the routes."""
    from paper_2406_08496_amd import synth
    from paper_2406_08496_amd.assign import Router, msa_switch

    inst = synth.regional()
    rng = np.random.default_rng(seed)
    base = inst.length.astype(np.float64) / inst.speed.astype(np.float64)
    o = np.ascontiguousarray(inst.meta["origin"], np.int32)
    d = np.ascontiguousarray(inst.meta["dest"], np.int32)
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=16, gpu=True)
    old = (inst.route_off, inst.route_edges)
    bufs = [np.empty(0, np.int32), np.empty(0, np.int32)]
    rows = []
    for n in range(1, n_iter + 1):
        cost = base * np.exp(rng.normal(0.0, 0.5, inst.n_edges))
        take = msa_switch(len(o), n, 0xA55)
        tm = {}
        new = r.routes(cost, o, d, old=old, take_new=take, timings=tm, out=bufs[n % 2])
        bufs[n % 2] = new[1].base if new[1].base is not None else new[1]
        rows.append({"n": n, "solve_ms": round(tm["route_solve"] * 1e3, 2), "fill_ms": round(tm["route_fill"] * 1e3, 2),
                     "moved": int(take.sum()), "route_entries": int(new[0][-1])})
        log("routing", json.dumps(rows[-1]))
        old = new
    later = rows[1:] or rows
    return {"workload": inst.name, "trips": len(o), "destinations": int(len(np.unique(d))),
            "iterations": rows,
            "mean_after_first_ms": {"solve": round(float(np.mean([x["solve_ms"] for x in later])), 2),
                                    "fill": round(float(np.mean([x["fill_ms"] for x in later])), 2)}}


def run_assignment(inst, n_iter):
    """MSA with the full simulation every iteration vs surrogate-assisted MSA
    (full simulation on iterations 1, 6, 11, ... and whenever the last
    simulation rejected the surrogate's estimate of its routes),
    same GPU; wall times include routing, simulation, loading and training.
    Agreement of the final edge travel times: flow-weighted mean relative
    difference, flow-weighted relative L2, and the relative difference of the
    total travel time (sum of exits x mean travel time)."""
    from paper_2406_08496_amd.assign import Assignment, agreement, edge_tt_errors

    a = Assignment(inst, n_bins=48, n_threads=16)
    a.progress = lambda r: log("plain", json.dumps(r))
    plain = a.run_plain(n_iter)
    log(f"plain MSA: {plain['wall_s']:.1f} s, timings {a.timings}")
    t_plain = {k: round(v, 2) for k, v in a.timings.items()}
    del a
    b = Assignment(inst, n_bins=48, n_threads=16)
    b.progress = lambda r: log("surrogate", json.dumps(r))
    sur = b.run_surrogate(n_iter)
    log(f"surrogate MSA: {sur['wall_s']:.1f} s, timings {b.timings}")
    t_sur = {k: round(v, 2) for k, v in b.timings.items()}
    w = plain["exits"].astype(np.float64)
    mean_rel, rel_l2 = edge_tt_errors(sur["tt"], plain["tt"], w)
    ttt_p = float((w * plain["tt"]).sum())
    ttt_s = float((sur["exits"].astype(np.float64) * sur["tt"]).sum())
    return {"iterations": n_iter, "plain_wall_s": plain["wall_s"], "surrogate_wall_s": sur["wall_s"],
            "speedup": plain["wall_s"] / sur["wall_s"], "full_simulations": {"plain": n_iter, "surrogate": sur["n_sim"]},
            "final_tt_mean_rel": mean_rel, "final_tt_rel_l2": rel_l2,
            "total_travel_time_rel": ttt_s / ttt_p - 1.0,
            "judge_errors": [h["judge_err"] for h in sur["hist"] if "judge_err" in h],
            "timings_s": {"plain": t_plain, "surrogate": t_sur},
            "router": "gpu"}


if __name__ == "__main__":
    main()
