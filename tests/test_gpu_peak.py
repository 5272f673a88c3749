"""Bit-exact parity at the peak of load, at full size and in the launch
shape the benchmark times (512 threads x 640 blocks, graphs of 64 steps).

The expected values are digests of the CPU oracle's full state and
statistics at sampled steps up to and past the demand peaks, written by
`tests/golden/make_peak_digests.py`, which calls only the oracle and the
seeded input generators.  The GPU library steps the same instance to the
same steps and its read-back must hash to the same digests: every vehicle's
status, edge, lane, cell, arrival step and the bit patterns of x and v, and
every per-edge statistic.  A mismatch names the array and the first
differing block of 2^16 trips or edges.

- regional: 2.82M trips; steps 7,200, 14,400, 19,136 (the step with the
  most vehicles on the road, 1.72M, where the benchmark's window starts),
  19,156 (the window's end) and 28,800 (the horizon);
- large: 9M trips, at the two demand peaks;
- batch: the 64-scenario batch in one context; two of its largest
  scenarios are compared (vehicles and statistics; the counters are
  batch-wide) through their peaks.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2406_08496_amd import synth

from test_gpu_parity import case

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from peak_digest import compare, digest  # noqa: E402

pytestmark = pytest.mark.gpu

BENCH_LAUNCH = (512, 640, 64)
DIGESTS = os.path.join(HERE, "golden", "peak_digests.json")


@pytest.fixture(scope="module")
def Sim():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_08496_amd.lpsim import Simulator

    return Simulator


@pytest.fixture(scope="module")
def table():
    with open(DIGESTS) as f:
        return json.load(f)


@pytest.mark.parametrize("workload", ["regional", "large"])
def test_peak_digests(Sim, table, workload):
    if workload not in table:
        pytest.skip(f"no oracle digests for {workload}")
    want = table[workload]
    inst = synth.regional() if workload == "regional" else synth.large()
    assert inst.n_trips == want["trips"] and inst.n_edges == want["edges"]
    gpu = Sim(n_bins=want["n_bins"])
    gpu.set_launch(*BENCH_LAUNCH)
    gpu.load(inst)
    done = 0
    for step in sorted(int(k) for k in want["checkpoints"]):
        gpu.step(step - done)
        done = step
        c = gpu.counters()
        case(workload, "digest at step", step, "active", c["active"], "waiting", c["waiting"])
        got = digest(gpu.vehicles(), gpu.edge_stats(), c)
        compare(got, want["checkpoints"][str(step)], f"{workload} step {step}")


def test_peak_digests_batch(Sim, table):
    names = sorted((k for k in table if k.startswith("batch:")), key=lambda k: int(k.split(":")[1]))
    if not names:
        pytest.skip("no oracle digests for the batch")
    insts = synth.batch_scenarios()
    gpu = Sim(n_bins=48)
    gpu.set_launch(*BENCH_LAUNCH)
    gpu.load_batch(insts)
    steps = sorted({int(s) for k in names for s in table[k]["checkpoints"]})
    done = 0
    for step in steps:
        gpu.step(step - done)
        done = step
        vg, sg = gpu.vehicles(), gpu.edge_stats()
        for k in names:
            want = table[k]["checkpoints"].get(str(step))
            if want is None:
                continue
            s = int(k.split(":")[1])
            t0, t1 = gpu.trip_off[s], gpu.trip_off[s + 1]
            e0, e1 = gpu.edge_off[s], gpu.edge_off[s + 1]
            assert t1 - t0 == table[k]["trips"] and e1 - e0 == table[k]["edges"]
            case("batch scenario", s, "digest at step", step)
            # the batch reports each scenario's trips with its own edge ids
            got = digest({n: vg[n][t0:t1] for n in vg}, {n: sg[n][e0:e1] for n in sg},
                         {n: 0 for n in want["counters"]})
            compare(got, want, f"{k} step {step}", counters=False)
