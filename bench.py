"""Benchmark: vehicle-steps per second of the LPSim vehicle update on one MI355X.

Workload (the paper's single-GPU regional case at its published size, on
synthetic stand-ins for the SF Bay network and SFCTA demand): planar road
graph of 225,150 nodes and 550,000 directed edges, 2,820,000 routed trips over
a two-peak 3 h morning profile, dt = 0.5 s, horizon 28,800 steps.

A "step" is one simulation time step of every vehicle (move, resolve, lane
change, commit).  value = vehicle-steps / s over the timed steps (a
vehicle-step is one vehicle active at the start of a step), inputs resident in
device memory.  The roofline entry prices the dominant kernel's measured
algorithmic bytes against the MI355X HBM peak; `cpu_baseline` times the plain
CPU oracle on a bounded prefix of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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
# id, claim word and request, 20; the departure requests' queue, trip and
# entry-window reads, which run in the same launch):
#   slot state read: meta, x, v (12) + the cached edge data the update needs:
#     lane offset, cells | look-ahead | next-edge-blocked, speed limit, next
#     lane offset (16)
#   slot state write: x, v, meta (12)
MOVE_FIXED_BYTES = 12 + 16 + 12

# HBM traffic of one k_move launch on this workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE: KiB per dispatch, mean over the 28,800
# launches), each scaled by what the same counter reads for a plain 1 GiB
# device copy (FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of them).
# Valid only for the workload and the kernel source it was taken on (sha256
# below); otherwise the bench reports null.  Commands and figures:
# profiles/k_move_regional_hbm_traffic.md
MOVE_TRAFFIC_WORKLOAD = "regional-225k-2.82M"
MOVE_TRAFFIC = {"kernels_sha256": "5161b11eed9ab4a33091ed24691d63b4cc3fe7214637d890c7ba81ac54bb816d",
                "fetch_kib": 29218.37, "write_kib": 16417.55, "fetch_scale": 2.0, "write_scale": 1.0}


def move_traffic_bytes(workload=MOVE_TRAFFIC_WORKLOAD):
    import hashlib

    if workload != MOVE_TRAFFIC_WORKLOAD:
        return None
    src = os.path.join(ROOT, "paper_2406_08496_amd", "csrc", "lpsim_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    t = MOVE_TRAFFIC
    if t["kernels_sha256"] != sha or t["fetch_kib"] is None:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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


def cpu_baseline(inst, n_bins, budget_s, plan=None):
    """The oracle as it is, single thread, from step 0 until the budget runs out."""
    import oracle

    o = oracle.OracleSim(n_bins=n_bins).load(inst)
    if plan is not None:
        o.set_signals(plan)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s and steps < inst.n_steps:
        o.step(100)
        steps += 100
    el = time.perf_counter() - t0
    c = o.counters()
    return {"value": c["vehicle_steps"] / el, "unit": "vehicle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"steps 0..{steps} of the same workload ({c['vehicle_steps']} vehicle-steps, "
                      f"{el:.1f} s, single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: full horizon)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--repeat", type=int, default=3,
                    help="timed runs of the same steps from the same state; the median is reported")
    ap.add_argument("--workload", default="regional")
    ap.add_argument("--block", type=int, default=512)
    ap.add_argument("--blocks", type=int, default=640)
    ap.add_argument("--graph-steps", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
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
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale the HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
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
    K = args.steps if args.steps is not None else horizon
    W = args.warmup
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
    tuned = None
    if args.autotune:
        # tune on a loaded state (a third of the horizon in), then rewind
        snap = sim.save_state()
        sim.step(horizon // 3)
        tuned = sim.autotune(n_steps=64)
        sim.restore_state(snap)
        log(f"autotuned: block {tuned['block_size']}, blocks {tuned['blocks']}")
        tuned = {"block": tuned["block_size"], "blocks": tuned["blocks"]}
    # warm-up steps (graph capture, caches), then rewind to step 0
    snap0 = sim.save_state()
    if W:
        sim.step(W, stream=stream)
        torch.cuda.synchronize()
    sim.restore_state(snap0)

    runs = []
    for r in range(max(1, args.repeat)):
        if r:
            sim.restore_state(snap0)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        t0 = time.perf_counter()
        sim.step(K, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs.append((ev0.elapsed_time(ev1), wall))
        log(f"run {r}: {runs[-1][0]:.1f} ms")
    ms, wall = sorted(runs)[len(runs) // 2]
    c = sim.counters()
    vsteps = c["vehicle_steps"]
    value = vsteps / (ms / 1e3)
    log(f"timed {K} steps: {ms:.1f} ms (wall {wall * 1e3:.1f} ms), {vsteps} vehicle-steps, "
        f"arrived {c['arrived']}/{n_trips}, active {c['active']}, watchdog {c['watchdog']}")

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
        "config": {"workload": name, "nodes": n_nodes, "edges": n_edges,
                   "trips": n_trips, "dt": 0.5, "horizon_steps": horizon,
                   "block": tuned["block"] if tuned else args.block,
                   "blocks": tuned["blocks"] if tuned else args.blocks, "graph_steps": args.graph_steps,
                   "signalised_nodes": plan.n_signals if plan is not None else 0},
        "trips_per_s": c["arrived"] / (ms / 1e3),
        "arrived": c["arrived"],
        "vehicle_steps": vsteps,
        "runs_ms": [round(x[0], 2) for x in runs],
    }

    if not args.no_roofline:
        # same K steps from the same state, kernels launched one by one with a
        # HIP event pair around each on the work stream
        sim.restore_state(snap0)
        sim.set_timing(True)
        sim.step(K, stream=stream)
        torch.cuda.synchronize()
        times = sim.kernel_times()
        c2 = sim.counters()
        sim.set_timing(False)
        dom = max(times, key=lambda k: times[k][0])
        alg_bytes = MOVE_FIXED_BYTES * c2["vehicle_steps"] + c2["scan_bytes"]
        mv_ms, mv_n = times["move"]
        achieved = alg_bytes / (mv_ms / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": "k_move", "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": move_traffic_bytes(name),
                           "bytes_per_launch": alg_bytes / max(mv_n, 1),
                           "avg_launch_us": mv_ms * 1e3 / max(mv_n, 1)}
        out["kernel_ms"] = {k: {"total_ms": v[0], "launches": v[1],
                                "avg_us": (v[0] * 1e3 / v[1]) if v[1] else None}
                            for k, v in times.items()}
        out["dominant_kernel"] = dom
        log("kernel times:", json.dumps(out["kernel_ms"]))

    if not args.no_mlp:
        out["surrogate_mlp"] = run_mlp(args.mlp_samples, 8192)
        log("surrogate perceptron:", json.dumps(out["surrogate_mlp"]))
    if not args.no_cpu_baseline and not batch:
        out["cpu_baseline"] = cpu_baseline(inst, n_bins, args.cpu_budget, plan)
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
    del a
    b = Assignment(inst, n_bins=48, n_threads=16)
    b.progress = lambda r: log("surrogate", json.dumps(r))
    sur = b.run_surrogate(n_iter)
    log(f"surrogate MSA: {sur['wall_s']:.1f} s, timings {b.timings}")
    w = plain["exits"].astype(np.float64)
    mean_rel, rel_l2 = edge_tt_errors(sur["tt"], plain["tt"], w)
    ttt_p = float((w * plain["tt"]).sum())
    ttt_s = float((sur["exits"].astype(np.float64) * sur["tt"]).sum())
    return {"iterations": n_iter, "plain_wall_s": plain["wall_s"], "surrogate_wall_s": sur["wall_s"],
            "speedup": plain["wall_s"] / sur["wall_s"], "full_simulations": {"plain": n_iter, "surrogate": sur["n_sim"]},
            "final_tt_mean_rel": mean_rel, "final_tt_rel_l2": rel_l2,
            "total_travel_time_rel": ttt_s / ttt_p - 1.0,
            "judge_errors": [h["judge_err"] for h in sur["hist"] if "judge_err" in h]}


if __name__ == "__main__":
    main()
