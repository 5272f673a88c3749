"""Write tests/golden/peak_digests.json: digests of the CPU oracle's full
state and statistics at sampled steps of the full-size workloads, up to and
past their peaks of load.

Only the oracle (its all-cores build, whose results equal the single-threaded
build's) and the seeded input generators are called; nothing comes from the
GPU library.  Each workload's entry is replaced, the others are kept:

    python tests/golden/make_peak_digests.py regional 7200,14400,28800
    python tests/golden/make_peak_digests.py large 12000,19200
    python tests/golden/make_peak_digests.py batch:63 4800,7200
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from paper_2406_08496_amd import synth  # noqa: E402
from peak_digest import digest  # noqa: E402

OUT = os.path.join(HERE, "peak_digests.json")


def instance(name):
    """(instance, n_bins) of a named workload; batch:s is scenario s of the
    64-scenario batch, run alone (a batched scenario equals its solo run)."""
    if name == "regional":
        return synth.regional(), 48
    if name == "large":
        return synth.large(), 60
    if name.startswith("batch:"):
        return synth.batch_scenarios()[int(name.split(":")[1])], 48
    raise SystemExit(f"unknown workload {name}")


def main():
    name, steps = sys.argv[1], sorted(int(s) for s in sys.argv[2].split(","))
    t0 = time.time()
    inst, n_bins = instance(name)
    print(f"{name}: {inst.n_nodes} nodes, {inst.n_edges} edges, {inst.n_trips} trips "
          f"(generated in {time.time() - t0:.0f} s)", flush=True)
    sim = oracle.OracleSim(parallel=True, n_bins=n_bins).load(inst)
    entry = {"n_bins": n_bins, "trips": inst.n_trips, "edges": inst.n_edges, "checkpoints": {}}
    done = 0
    t0 = time.time()
    for target in steps:
        while done < target:
            n = min(600, target - done)
            sim.step(n)
            done += n
            c = sim.counters()
            print(f"  step {done}: active {c['active']}, waiting {c['waiting']}, arrived {c['arrived']}, "
                  f"{time.time() - t0:.0f} s", flush=True)
        assert not sim.invariant_broken
        entry["checkpoints"][str(target)] = digest(sim.vehicles(), sim.edge_stats(), sim.counters())
        print(f"  digest at step {target}", flush=True)
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    table[name] = entry
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"wrote {name} to {OUT} ({time.time() - t0:.0f} s of simulation)", flush=True)


if __name__ == "__main__":
    main()
