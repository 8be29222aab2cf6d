"""Autotuner of the batched solve: workgroup size and sweeps per hipGraph
replay, chosen per size class by timing candidates on the device, cached in
a JSON file keyed by GPU architecture and size class.

A replay of S sweeps ends with the stop decision, so S trades host round
trips (fewer for large S) against sweeps done after a problem has already
met the tolerance (up to S - 1).  The tuner keeps the smallest S whose
steady-state time per sweep is within 2 % of the best.

The size class of a batch is (number of problems, log2 bucket of the total
free nodes, largest grid side); batches of one class share the choice.
"""
from __future__ import annotations

import json
import math
import os

import torch

BLOCKS = (128, 256, 512)
SWEEPS_PER_GRAPH = (8, 16, 32, 64)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def arch_name(device=0):
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name)


def size_class(batch):
    total = sum(batch.n_free)
    side = max(max(p["n"]) for p in batch.problems)
    return f"n{batch.n}-free2^{int(math.log2(max(total, 1)))}-side{side}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(batch, cache_path=DEFAULT_CACHE, replays=2, force=False):
    """Return (block, sweeps_per_graph) for this batch, timing the candidates
    unless the cache already holds its (arch, size class)."""
    key = f"{arch_name()}|{size_class(batch)}"
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return int(c["block"]), int(c["sweeps_per_graph"])
    results = []
    for block in BLOCKS:
        results.append((batch.time_config(block, 16, replays=replays), block, 16))
    block = min(results)[1]
    for S in SWEEPS_PER_GRAPH:
        if S != 16:
            results.append((batch.time_config(block, S, replays=replays), block, S))
    mine = [r for r in results if r[1] == block]
    best_t = min(r[0] for r in mine)
    t, block, S = min((r for r in mine if r[0] <= 1.02 * best_t), key=lambda r: r[2])
    if cache_path:
        cache[key] = {"block": block, "sweeps_per_graph": S, "seconds_per_sweep": t,
                      "candidates": [{"block": b, "sweeps_per_graph": s, "seconds_per_sweep": x}
                                     for x, b, s in results]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return block, S
