"""Digests of a simulation's full state and statistics, for comparing long
runs at sampled steps without storing the arrays.

Each array is hashed whole (SHA-256 of its bytes, in trip or edge order) and
in chunks of 2^16 elements (12 hex digits each), so a mismatch names the
array and the trip or edge range where it starts.  The same function hashes
the oracle's read-back (when the stored values are written) and the GPU
library's read-back (in the tests); it only hashes, it computes nothing of
the method.
"""
from __future__ import annotations

import hashlib

import numpy as np

VEHICLE_KEYS = ("status", "edge", "lane", "cell", "x", "v", "arrival_step")
STAT_KEYS = ("tt_sum", "n_exits", "inflow_bin", "exits_bin", "tt_bin", "occ_bin")
COUNTER_KEYS = ("step", "active", "waiting", "arrived", "vehicle_steps", "transfers",
                "departures", "claims_lost", "lc_attempts", "lc_accepts", "watchdog")
CHUNK = 1 << 16

# the dtype each array is hashed in (the read-back dtypes of both sides)
DTYPES = {"status": np.uint8, "edge": np.int32, "lane": np.uint8, "cell": np.int32,
          "x": np.float32, "v": np.float32, "arrival_step": np.int32,
          "tt_sum": np.int64, "n_exits": np.int32, "inflow_bin": np.int32,
          "exits_bin": np.int32, "tt_bin": np.int64, "occ_bin": np.int64}


def _array_digest(a, key):
    a = np.ascontiguousarray(a, DTYPES[key])
    rows = a.reshape(a.shape[0], -1)
    whole = hashlib.sha256(rows.tobytes()).hexdigest()
    chunks = [hashlib.sha256(rows[i:i + CHUNK].tobytes()).hexdigest()[:12]
              for i in range(0, rows.shape[0], CHUNK)]
    return {"sha256": whole, "chunks": chunks}


def digest(vehicles, stats, counters):
    """{array: {sha256, chunks}} for the vehicle and statistics arrays, plus
    the counters as plain integers."""
    out = {"vehicles": {k: _array_digest(vehicles[k], k) for k in VEHICLE_KEYS},
           "stats": {k: _array_digest(stats[k], k) for k in STAT_KEYS},
           "counters": {k: int(counters[k]) for k in COUNTER_KEYS}}
    return out


def compare(got, want, where="", counters=True):
    """Raise AssertionError naming the first differing counter, array and
    chunk (chunk c covers elements [c * 2^16, (c + 1) * 2^16)).  counters:
    False skips the run-wide counters (one scenario of a batch has none of
    its own)."""
    for k in COUNTER_KEYS if counters else ():
        if got["counters"][k] != want["counters"][k]:
            raise AssertionError(f"{where}: counter {k}: got {got['counters'][k]} want {want['counters'][k]}")
    for part in ("vehicles", "stats"):
        for k, w in want[part].items():
            g = got[part][k]
            if g["sha256"] != w["sha256"]:
                bad = [i for i, (a, b) in enumerate(zip(g["chunks"], w["chunks"])) if a != b]
                raise AssertionError(f"{where}: {part} {k} differs; first differing chunk "
                                     f"{bad[:4]} of {len(w['chunks'])} (2^16 elements each)")
