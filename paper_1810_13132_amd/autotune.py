"""Launch-shape autotuner for batched steps.

Times whole batch steps for each candidate (scan tile, estimate tile,
workgroups per CU) on the caller's inputs (one slice or several) with HIP
events and keeps the fastest.  Tuning runs real steps, so it should be given a scratch batch with
the production shapes (or accept that the timed steps advance the windows).
Results can be cached in a JSON file keyed by the device and a batch
signature (per-sketch m, g, k, layout and log2 buckets of the step sizes).
"""
import json
import math
import os

import torch

DEFAULT_CANDIDATES = [(st, et, bpc) for st in (2048, 8192, 32768) for et in (16, 64, 256) for bpc in (4, 8, 16)]


def signature(params, n_pairs, n_hosts) -> str:
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", dev.name)
    parts = [f"{p['m']}:{p['g']}:{p['k']}:{p.get('layout', 'fast')}:{int(math.log2(max(a, 1)))}:"
             f"{int(math.log2(max(b, 1)))}" for p, a, b in zip(params, n_pairs, n_hosts)]
    return arch + "|" + ",".join(parts)


def time_steps(batch, pairs, hosts, outs, reps: int) -> float:
    """ms per step over reps passes through the given slices; pairs is one
    step's per-sketch pair tensors or a list of such steps (slices whose
    record runs and plane occupancy differ time differently)."""
    steps = pairs if pairs and isinstance(pairs[0], (list, tuple)) else [pairs]
    batch.step(steps[0], hosts, outs)  # warm (and capture the graph)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        for step in steps:
            batch.step(step, hosts, outs)
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / (reps * len(steps))


def tune(batch, pairs, hosts, outs, candidates=None, reps: int = 3, cache_path: str = None, key: str = None):
    """Return (best tuning dict, {candidate: ms per step}); applies the best to the batch."""
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key and key in cache:
        best = cache[key]["best"]
        batch.set_tuning(best["scan_tile"], best["est_tile"], best["blocks_per_cu"], True)
        return best, cache[key]["timings"]
    timings = {}
    for st, et, bpc in candidates or DEFAULT_CANDIDATES:
        batch.set_tuning(st, et, bpc, True)
        timings[f"{st},{et},{bpc}"] = time_steps(batch, pairs, hosts, outs, reps)
    best_key = min(timings, key=timings.get)
    st, et, bpc = (int(v) for v in best_key.split(","))
    best = {"scan_tile": st, "est_tile": et, "blocks_per_cu": bpc}
    batch.set_tuning(st, et, bpc, True)
    if cache_path and key:
        cache[key] = {"best": best, "timings": timings}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best, timings
