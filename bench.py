#!/usr/bin/env python
"""Throughput of the VBDR per-slice hot path on one MI355X.

One step = one time slice of the line-rate workload: scan its 2^26 (aip, bip)
pairs into the BDR pool (m = 2^26, g = 1024), advance the window (k = 60),
and estimate every host active in the window (of 2^20 hosts).  Pairs and
host lists are resident in HBM before timing starts.  The timed steps are
slices k .. k+K-1 by default: the window is full and the pool has aged
through k untimed slices (its steady state).  A secondary figure
(`young_pool`) times slices W .. W+K-1 of a fresh pool.

    python bench.py [--steps K] [--warmup W] [--layout small|fast|packed]
                    [--workload line_rate|tiny|batched|stress]

Prints one JSON line.  value = IP pairs per second through whole steps.
The aging slices scan and advance only, so under a profiler every estimate
launch belongs to a full-window step (warm-up or timed).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IP pairs/s scanned + hosts estimated/s at 1 GPU; learned vs plain RMS rel. error"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")
CSRC = os.path.join(ROOT, "paper_1810_13132_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind, w, layout, L, n_hosts, dr_bits=8):
    """Bytes a launch must move at minimum (per unit x units).  For the packed
    layout L is its recorder count Lc and dr_bits its DR width z."""
    if kind == "scan":  # pair read + one state update (fast: 4 B word read-modify-write; small/packed: 1 B store)
        return w.pairs_per_slice * (16 if layout == "fast" else 9)
    if kind == "advance":  # every DR read and written, register written; fast: bsLBP1 bits read and cleared
        per = 2 * L * dr_bits / 8 + 1 + (2 * L / 8 if layout == "fast" else 0)
        return w.m * per
    if kind == "estimate":  # g register gathers + host id + estimate
        return n_hosts * (w.g + 8)
    raise ValueError(kind)


def tiled_design_bytes(w, n_hosts, narrow=False):
    """HBM bytes the LDS-tiled estimate moves by construction: each (host, i)
    record written and read once (8 B), each (tile, host) partial sum written
    and read once (8 B, or 4 B in the 16-bit form the estimate takes when
    registers 0..2 are under 1/64 of the pool), host id and estimate (8 B).
    Tiles: at most 256, of 2^s registers with s >= 12 the smallest that
    covers the padded pool."""
    mstride = (w.m + 4095) // 4096 * 4096
    s = 12
    while (1 << s) * 256 < mstride:
        s += 1
    nt = (mstride + (1 << s) - 1) >> s
    return n_hosts * (8 * w.g + (4 if narrow else 8) * nt + 8)


# gfx950 L2: 8 XCDs x 16 channels, one tag lookup per channel per clock at 2.4 GHz.
# A random 1-byte register gather that misses L1 costs one such request.
L2_REQ_PEAK = 8 * 16 * 2.4e9


def traffic_from_counters(kernel_name, n_launch_units):
    """HBM bytes per call of a hot-path stage (all kernels it launches) from
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs, if they were taken on the
    current kernel sources; else None."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("src_sha") != kernel_source_hash():
        return None
    k = c.get("kernels", {}).get(kernel_name)
    if not k:
        return None
    b = (k["fetch_kib"] * c["fetch_scale"] + k["write_kib"] * c["write_scale"]) * 1024.0
    if k.get("units_per_call"):  # per-call work that varies (hosts estimated): scale to this run's units
        b *= n_launch_units / k["units_per_call"]
    return b


def cpu_baseline(w, layout, slice0, hosts_sample, n_active, Lc=0):
    """Time the CPU oracle (single thread, as it stands) on a bounded sample."""
    import numpy as np
    from oracle import oracle
    code = {"fast": oracle.GFAST, "small": oracle.GSMALL, "packed": oracle.GPACKED}[layout]
    S = min(len(slice0), 1 << 22)
    t0 = time.perf_counter()
    osk = oracle.Sketch(w.m, w.g, w.k, w.seed, code, Lc=Lc)
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    osk.scan(slice0[:S])
    t_scan = time.perf_counter() - t0
    t0 = time.perf_counter()
    osk.advance()
    t_adv = time.perf_counter() - t0
    t0 = time.perf_counter()
    osk.estimate(hosts_sample)
    t_est = time.perf_counter() - t0
    step = t_scan * (w.pairs_per_slice / S) + t_adv + t_est * (n_active / len(hosts_sample))
    del osk
    return {"value": w.pairs_per_slice / step, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"one slice: scan of the first {S} of {w.pairs_per_slice} pairs, one full advance of "
                      f"{w.m} BDRs, estimate of {len(hosts_sample)} of {n_active} active hosts; scaled to a "
                      f"whole step (scan x{w.pairs_per_slice // S}, estimate x{n_active / len(hosts_sample):.0f})",
            "seconds": {"create": round(t_create, 3), "scan": round(t_scan, 3), "advance": round(t_adv, 3),
                        "estimate": round(t_est, 3)}}


def _oracle_step_worker(job):
    """One process of the all-cores baseline: the single-threaded oracle on
    the same bounded sample as cpu_baseline; returns its scaled step time."""
    import numpy as np
    from oracle import oracle
    w_m, w_g, w_k, seed, code, Lc, pairs, hosts, scale_scan, scale_est = job
    t0 = time.perf_counter()
    osk = oracle.Sketch(w_m, w_g, w_k, seed, code, Lc=Lc)
    t1 = time.perf_counter()
    osk.scan(pairs)
    t2 = time.perf_counter()
    osk.advance()
    t3 = time.perf_counter()
    osk.estimate(hosts)
    t4 = time.perf_counter()
    del osk
    return (t2 - t1) * scale_scan + (t3 - t2) + (t4 - t3) * scale_est, t4 - t0


def cpu_baseline_all_cores(w, layout, slice0, hosts_sample, n_active, Lc=0, max_workers=16):
    """The same oracle sample run by one single-threaded process per host core
    at once (at most max_workers, the host share of one GPU): the aggregate
    rate of the CPU doing independent steps in parallel.  The oracle itself
    stays single-threaded."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import oracle
    code = {"fast": oracle.GFAST, "small": oracle.GSMALL, "packed": oracle.GPACKED}[layout]
    n = max(1, min(max_workers, os.cpu_count() or 1))
    S = min(len(slice0), 1 << 22)
    job = (w.m, w.g, w.k, w.seed, code, Lc, slice0[:S].copy(), hosts_sample, w.pairs_per_slice / S,
           n_active / len(hosts_sample))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(n, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_step_worker, [job] * n))
    wall = time.perf_counter() - t0
    step = max(r[0] for r in res)
    return {"value": n * w.pairs_per_slice / step, "unit": "pairs/s", "cores": n, "kind": "oracle",
            "sample": f"{n} single-threaded oracle processes at once, each on the cpu_baseline sample (scan of "
                      f"{S} pairs, one advance of {w.m} BDRs, {len(hosts_sample)} host estimates), scaled to a "
                      f"step; value = processes x pairs per step / the slowest process's scaled step",
            "seconds_wall": round(wall, 2)}


def scan_roofline(w, layout, ms):
    b = algorithmic_bytes("scan", w, layout, 0, 0)
    rate = b / (ms * 1e-3) / 1e9
    return {"achieved": round(rate, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(rate / HBM_PEAK_GBS, 4)}


def learned_accuracy():
    """Plain vs learned RMS relative error, and both estimators' hosts/s, on
    the evaluation streams (seeds 100..109) of each workload shape a network
    was trained on: the tiny workload (all ten seeds) and the mid workload
    (seeds 100..102); None when no trained weights are present."""
    from paper_1810_13132_amd import learn, synth
    out = {}
    for name, path, w, seeds in (("tiny", learn.DEFAULT_WEIGHTS, synth.TINY, range(100, 110)),
                                 ("mid", learn.MID_WEIGHTS, synth.MID, range(100, 103))):
        if not os.path.exists(path):
            continue
        params, lo, hi, meta = learn.load(path)
        res = learn.evaluate(params, lo, hi, eval_seeds=seeds, w=w)
        res["workload"] = (f"{w.name} ({w.hosts} hosts, {w.pairs_per_slice} pairs/slice, m={w.m}, g={w.g}, "
                           f"k={w.k}), eval seeds {min(seeds)}..{max(seeds)}")
        res["trained_on"] = meta.get("train_seeds")
        out[name] = res
    return out or None


def run_batched(args):
    """32 independent edge-router streams stepped together: persistent kernels,
    graph replay, launch shape picked by the autotuner on a scratch batch."""
    import numpy as np
    import torch
    from paper_1810_13132_amd import autotune, synth, vbdr
    torch.cuda.set_device(0)
    ws = synth.batched_workloads()
    K, W = args.steps, args.warmup
    params = [dict(m=w.m, g=w.g, k=w.k, hash_seed=w.seed, layout=args.layout) for w in ws]
    streams = [synth.Stream(w) for w in ws]
    pairs = [[vbdr.to_device_u32(st.slice(t).reshape(-1)) for st in streams] for t in range(W + K)]
    log(f"batched: {len(ws)} streams, {sum(w.pairs_per_slice for w in ws)} pairs per step generated")
    hosts = [vbdr.to_device_u32(st.aip) for st in streams]
    outs = [torch.empty(h.numel(), dtype=torch.float32, device="cuda") for h in hosts]
    scratch = vbdr.Batch(params)
    best, timings = autotune.tune(scratch, pairs[:min(4, len(pairs))], hosts, outs, reps=1)
    scratch.close()
    log(f"autotuned: {best}")
    bt = vbdr.Batch(params)
    bt.set_tuning(best["scan_tile"], best["est_tile"], best["blocks_per_cu"], True)
    for t in range(W):
        bt.step(pairs[t], hosts, outs)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    ev[0].record()
    for t in range(W, W + K):
        bt.step(pairs[t], hosts, outs)
    ev[1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_pairs = sum(w.pairs_per_slice for w in ws)
    n_hosts = sum(h.numel() for h in hosts)
    res = {"metric": METRIC, "value": n_pairs * K / elapsed, "unit": "pairs/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "batched", "sketches": len(ws), "pairs_per_step": n_pairs,
                      "hosts_per_step": n_hosts, "layout": args.layout, "tuning": best},
           "hosts_per_s": n_hosts * K / elapsed, "graph_ms_per_step": ev[0].elapsed_time(ev[1]) / K,
           "autotune_ms_per_step": timings}
    print(json.dumps(res), flush=True)


def run_stress(args):
    """Skewed contention: 16 planted superspreaders (10^6..10^7 opposite hosts)
    among 2^24 hosts, 2^27 pairs per slice into m = 2^24 BDRs (g = 2048,
    k = 128).  Each step estimates the superspreaders plus 2^16 sampled
    background hosts; errors are reported per group over the window of the
    last timed step.  The timed steps start at slice k (first_slice): the
    slices before it fill the window untimed (scan and advance only)."""
    import numpy as np
    import torch
    from paper_1810_13132_amd import learn, synth, vbdr
    torch.cuda.set_device(0)
    w = synth.STRESS
    K, W = args.steps, args.warmup
    S0 = args.first_slice if args.first_slice is not None else max(w.k, W)
    st = synth.Stream(w)
    rng = np.random.default_rng(5)
    heavy = np.arange(w.n_heavy)
    background = rng.choice(np.arange(w.n_heavy, w.hosts), size=1 << 16, replace=False)
    sel = np.concatenate([heavy, background])
    hosts = vbdr.to_device_u32(st.aip[sel])
    host_keys = torch.from_numpy(st.aip[sel].astype(np.int64)).cuda()
    sk = vbdr.Sketch(w.m, w.g, w.k, w.seed, args.layout)
    out = torch.empty(len(sel), dtype=torch.float32, device="cuda")
    seen_keys = []
    times = []
    t0 = time.time()
    for t in range(S0 + K):
        pd = vbdr.to_device_u32(st.slice(t).reshape(-1))
        p = pd.view(-1, 2).to(torch.int64) & 0xFFFFFFFF
        keep = torch.isin(p[:, 0], host_keys)
        seen_keys.append(torch.unique((p[keep, 0] << 32) | p[keep, 1]))
        seen_keys = seen_keys[-w.k:]
        del p, keep
        torch.cuda.synchronize()
        if t < S0 - W:  # aging: the state only
            sk.scan_slice(pd)
            sk.advance_slice()
            if t % 8 == 0:
                log(f"stress slice {t} (aging, {time.time() - t0:.0f}s)")
            del pd
            continue
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sk.scan_slice(pd)
        sk.advance_slice()
        sk.estimate(hosts, out)
        b.record()
        b.synchronize()
        if t >= S0:
            times.append(a.elapsed_time(b))
        log(f"stress slice {t}: {a.elapsed_time(b):.2f} ms" + ("" if t >= S0 else " (warm-up)"))
        del pd
    truth = learn.window_truth(seen_keys[-w.k:], host_keys)
    est = out.to(torch.float64)
    # super-point detection at a threshold between the planted (>= 10^6) and background (<= 10^4) populations
    thr = 1e5
    found, _, n_found = vbdr.select_hosts(out, hosts, thr)
    found = set(found.cpu().numpy().view(np.uint32).tolist())
    real = set(st.aip[sel][(truth >= thr).cpu().numpy()].tolist())
    detect = {"threshold": thr, "selected": n_found, "true_positives": len(found & real),
              "precision": len(found & real) / max(len(found), 1), "recall": len(found & real) / max(len(real), 1)}
    ms = float(np.mean(times))
    res = {"metric": METRIC, "value": w.pairs_per_slice / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": "stress", "hosts": w.hosts, "pairs_per_slice": w.pairs_per_slice, "m": w.m,
                      "g": w.g, "k": w.k, "layout": args.layout, "estimated_hosts": len(sel),
                      "first_timed_slice": S0, "window_full": S0 >= w.k - 1},
           "rms_rel_superspreaders": learn.rms_rel(est[:w.n_heavy], truth[:w.n_heavy]),
           "rms_rel_background": learn.rms_rel(est[w.n_heavy:], truth[w.n_heavy:]),
           "detection": detect,
           "superspreader_truth": [int(v) for v in truth[:w.n_heavy].cpu()],
           "superspreader_estimate": [float(v) for v in est[:w.n_heavy].cpu()],
           "slices_in_window": min(S0 + K, w.k)}
    # the pool's own HyperLogLog estimate: the distinct pairs in the window
    hist = sk.registers()[1].astype(np.float64)
    alpha = 0.7213 / (1 + 1.079 / w.m)
    em = alpha * w.m * w.m / float(np.sum(hist * np.exp2(-np.arange(len(hist)))))
    if em <= 2.5 * w.m and hist[0] > 0:
        em = w.m * math.log(w.m / hist[0])
    res["pool_distinct_pairs_estimate"] = em
    if os.path.exists(learn.STRESS_WEIGHTS):
        # the stress-shape network (trained on synthetic stress windows) on the real stream's last window
        params, lo, hi, meta = learn.load(learn.STRESS_WEIGHTS)
        mlp = vbdr.MLP(params, lo, hi, meta.get("plain_above"))
        lest, fb = sk.estimate_learned(mlp, hosts, with_fallback=True)
        lest = lest.to(torch.float64)

        def rate(fn):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                fn()
            b.record()
            b.synchronize()
            return len(sel) * 5 / (a.elapsed_time(b) * 1e-3)

        res["learned"] = {
            "rms_rel_superspreaders": learn.rms_rel(lest[:w.n_heavy], truth[:w.n_heavy]),
            "rms_rel_background": learn.rms_rel(lest[w.n_heavy:], truth[w.n_heavy:]),
            "fallback_frac": float((fb == 1).float().mean()),
            "kept_plain_frac": float((fb == 2).float().mean()),
            "plain_above": meta.get("plain_above"),
            "hosts_per_s_plain": rate(lambda: sk.estimate(hosts, out)),
            "hosts_per_s_learned": rate(lambda: sk.estimate_learned(mlp, hosts)),
            "weights": "paper_1810_13132_amd/weights/mlp_stress.npz",
            "trained_on": meta.get("workload", "stress") + " synthetic windows " + str(meta.get("train_seeds"))}
        mlp.close()
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--layout", default="small", choices=["small", "fast", "packed"])
    ap.add_argument("--packed-lc", type=int, default=16,
                    help="recorders per BDR of the packed layout (LBP1 values above it are recorded at it)")
    ap.add_argument("--workload", default="line_rate", choices=["line_rate", "tiny", "batched", "stress"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the learned-vs-plain accuracy evaluation (profiling runs)")
    ap.add_argument("--overlap", action="store_true",
                    help="scan each slice on a second stream while the previous window is estimated")
    ap.add_argument("--first-slice", type=int, default=None,
                    help="first timed slice (default: k, or later if the young-pool steps need room); the "
                         "slices before it age the pool untimed")
    ap.add_argument("--no-young", action="store_true",
                    help="skip the secondary measurement on the young pool (slices warmup..warmup+steps-1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for rocprofv3 byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1810_13132_amd import synth, vbdr

    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "stress":
        return run_stress(args)
    w = synth.LINE_RATE if args.workload == "line_rate" else synth.TINY
    K, W = args.steps, args.warmup
    young = not args.no_young
    # first timed slice of the steady-state measurement: the window of k slices
    # is full from the close of slice k - 1 on; the pool before it is aged by
    # untimed slices (the stream is counter-based and stationary, so slices
    # past the workload's nominal count are the same workload)
    S0 = args.first_slice if args.first_slice is not None else max(w.k, (W + K if young else 0) + W)
    if S0 < W or (young and S0 < 2 * W + K):
        raise SystemExit("--first-slice leaves no room for the warm-up (and the young-pool steps)")
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    Lc = args.packed_lc if args.layout == "packed" else 0
    sk = vbdr.Sketch(w.m, w.g, w.k, w.seed, args.layout, Lc=Lc)
    L = sk.Lc
    info = sk.info()

    # ---- inputs: generated on the host; the slices of timed and warm-up steps
    # are resident in HBM before their timing starts, aging slices are scanned
    # as they are generated
    st = synth.Stream(w)
    hosts_all = st.aip
    resident = {}  # slice -> (pairs, active hosts, their count)
    in_window = np.zeros(w.hosts, dtype=np.int32)  # slices of the last k with pairs of the host
    window = []
    buf = np.empty((w.pairs_per_slice, 2), dtype=np.uint32)
    slice0 = None
    n_apply = 3 if info.scan_deferred else 0  # extra slices for the record-apply measurement
    t0 = time.time()

    def generate(t, keep):
        nonlocal slice0
        counts = np.zeros(w.hosts, dtype=np.uint32)
        st.slice(t, host_pairs=counts, out=buf)
        act = counts > 0
        in_window[act] += 1
        window.append(act)
        if len(window) > w.k:
            in_window[window.pop(0)] -= 1
        pd = vbdr.to_device_u32(buf.reshape(-1), dev)
        if t == S0 and not args.no_cpu_baseline:
            slice0 = buf.copy()
        if keep:
            hosts = np.nonzero(in_window)[0]
            resident[t] = (pd, vbdr.to_device_u32(hosts_all[hosts], dev), len(hosts))
        return pd

    main = torch.cuda.current_stream()
    side = torch.cuda.Stream() if args.overlap else main
    adv_done = [None]

    # Slice i's scan only needs slice i-1's advance (which drains the record
    # runs), not its estimate: with --overlap the scan runs on a second stream
    # of default priority while the main stream estimates the previous window;
    # the advance then waits for both.  Measured 1 % faster at the line-rate
    # workload (the two compete for the memory system), so the default keeps
    # one stream and per-stage times that are not stretched by the overlap.
    def step(i, out, e=None):
        pairs, hosts, _ = resident[i]
        if side is not main and adv_done[0] is not None:
            side.wait_event(adv_done[0])
        if e:
            e[0].record(side)
        sk.scan_slice(pairs, stream=side)
        if e:
            e[1].record(side)
        if side is not main:
            scanned = torch.cuda.Event()
            scanned.record(side)
            main.wait_event(scanned)
        if e:
            e[2].record(main)
        sk.advance_slice(stream=main)
        if e:
            e[3].record(main)
        adv_done[0] = torch.cuda.Event()
        adv_done[0].record(main)
        sk.estimate(hosts, out, stream=main)
        if e:
            e[4].record(main)

    def measure(first):
        """W warm-up steps, then K timed steps from slice `first` on."""
        outs = {i: torch.empty(resident[i][2], dtype=torch.float32, device=dev) for i in range(first - W, first + K)}
        for i in range(first - W, first):
            step(i, outs[i])
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
        t_start = time.perf_counter()
        for j in range(K):
            step(first + j, outs[first + j], ev[j])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kms = {"scan": [], "advance": [], "estimate": []}
        for e in ev:
            kms["scan"].append(e[0].elapsed_time(e[1]))
            kms["advance"].append(e[2].elapsed_time(e[3]))
            kms["estimate"].append(e[3].elapsed_time(e[4]))
        for i in range(first - W, first + K):
            del resident[i]
        return elapsed, kms, [resident_n[i] for i in range(first, first + K)]

    resident_n = {}
    n_first = 0
    res_young = None
    if young:
        for t in range(W + K):
            generate(t, True)
            resident_n[t] = resident[t][2]
        el, kms_y, act_y = measure(W)
        res_young = {"first_timed_slice": W, "ms_per_step": el * 1e3 / K,
                     "kernel_ms": {k_: round(float(np.mean(v)), 4) for k_, v in kms_y.items()},
                     "active_hosts_per_step": int(np.mean(act_y))}
        log(f"young pool (slices {W}..{W + K - 1}): {el * 1e3 / K:.3f} ms/step")
        n_first = W + K
    for t in range(n_first, S0 + K + n_apply):
        keep = t >= S0 - W
        pd = generate(t, keep)
        if keep:
            resident_n[t] = resident[t][2]
        else:  # aging: the state only, no estimate
            sk.scan_slice(pd)
            sk.advance_slice()
        del pd
        if t % 8 == 0 or keep:
            log(f"slice {t}: generated ({time.time() - t0:.1f}s), {int(np.count_nonzero(in_window))} hosts in window"
                + ("" if keep else " (aging)"))
    torch.cuda.synchronize()
    elapsed, kms, timed_active = measure(S0)
    log(f"timed {K} steps from slice {S0} in {elapsed:.3f}s")
    # the width of the tiled estimate's per-tile sums in the last timed step
    pool_hist = sk.registers()[1]
    low_regs = int(pool_hist[0] + pool_hist[1] + pool_hist[2])
    narrow_sums = bool(64 * low_regs < w.m)

    # The deferred scan's updates are applied by the next advance, from LDS:
    # that share of the advance belongs to the scan stage.  Measured on the
    # aged pool as the advance after a full slice's records minus the advance
    # after an empty slice, alternating.
    apply_ms = None
    if n_apply:
        ea = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_apply)]
        for j in range(n_apply):
            pairs = resident[S0 + K + j][0]
            sk.scan_slice(pairs)
            ea[j][0].record()
            sk.advance_slice()
            ea[j][1].record()
            ea[j][2].record()
            sk.advance_slice()
            ea[j][3].record()
        torch.cuda.synchronize()
        with_rec = [e[0].elapsed_time(e[1]) for e in ea]
        empty = [e[2].elapsed_time(e[3]) for e in ea]
        apply_ms = max(float(np.mean(with_rec) - np.mean(empty)), 0.0)
        log(f"advance with records {np.mean(with_rec):.4f} ms, after an empty slice {np.mean(empty):.4f} ms")
        resident.clear()

    avg = {k_: float(np.mean(v)) for k_, v in kms.items()}
    ms_per_step = elapsed * 1e3 / K
    value = w.pairs_per_slice * K / elapsed

    dom = max(avg, key=avg.get)
    units = float(np.mean(timed_active))
    alg = algorithmic_bytes(dom, w, args.layout, L, units, sk.dr_bits)
    achieved = alg / (avg[dom] * 1e-3) / 1e9
    info = sk.info()
    adv = "k_advance_packed" if args.layout == "packed" else "k_advance_defer" if info.scan_deferred else "k_advance"
    kernels = {"scan": "k_scan_defer" if info.scan_deferred else "k_scan",
               "advance": adv + " + k_hist_reset",
               "estimate": ("k_est_tile_clear + k_est_tile_bin + k_est_tile_gather + k_est_tile_wide + k_est_tile_final"
                            if info.est_tiled else
                            "k_estimate_part + k_estimate_final" if info.est_parts > 1 else "k_estimate")}
    traffic = traffic_from_counters(f"{dom}:{args.layout}:{w.name}", units)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernels[dom],
                "algorithmic_bytes_per_launch": alg}
    if dom == "estimate" and info.est_tiled:
        # the tiled estimate trades L2 gathers for streamed records and per-tile partial sums
        b = tiled_design_bytes(w, units, narrow_sums)
        rate = b / (avg["estimate"] * 1e-3) / 1e9
        roofline["design_bytes"] = {"per_launch": b, "achieved": round(rate, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(rate / HBM_PEAK_GBS, 4),
                                    "partial_sums": "16-bit" if narrow_sums else "32-bit",
                                    "pool_registers_0_to_2": round(low_regs / w.m, 5)}
    elif dom == "estimate":
        # the estimate moves few bytes; its limit is the L2 request rate of g random gathers per host
        gathers = units * w.g / (avg["estimate"] * 1e-3)
        roofline["l2_requests"] = {"achieved": gathers, "peak": L2_REQ_PEAK, "unit": "requests/s",
                                   "frac": round(gathers / L2_REQ_PEAK, 4)}

    res = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": w.name, "overlap": bool(args.overlap), "pairs_per_slice": w.pairs_per_slice,
                   "hosts": w.hosts, "m": w.m,
                   "g": w.g, "k": w.k, "layout": args.layout, "active_hosts_per_step": int(units),
                   **({"Lc": sk.Lc, "dr_bits": sk.dr_bits} if args.layout == "packed" else {}),
                   "first_timed_slice": S0, "window_full": S0 >= w.k - 1,
                   "state_bytes": int(info.state_bytes), "window_state_bytes": int(info.window_state_bytes),
                   "workspace_bytes": int(info.workspace_bytes)},
        "hosts_per_s": float(np.sum(timed_active) / (np.sum(kms["estimate"]) * 1e-3)),
        "scan_pairs_per_s": w.pairs_per_slice / (avg["scan"] * 1e-3),
        # the scan step against the HBM peak: algorithmic bytes per pair (pair + state update)
        "scan_roofline": scan_roofline(w, args.layout, avg["scan"]),
        "kernel_ms": {k: round(v, 4) for k, v in avg.items()},
        "roofline": roofline,
    }
    if apply_ms is not None:
        # deferred scans: the scan stage is the record-writing kernel plus the
        # advance's share that applies the records
        res["scan_apply_ms"] = round(apply_ms, 4)
        res["scan_with_apply_pairs_per_s"] = w.pairs_per_slice / ((avg["scan"] + apply_ms) * 1e-3)
        res["scan_with_apply_roofline"] = scan_roofline(w, args.layout, avg["scan"] + apply_ms)
    if res_young:
        res["young_pool"] = res_young
    acc = None if args.no_accuracy else learned_accuracy()
    if acc:
        res["accuracy"] = acc
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calibration_copy_bytes"] = src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(0)
        act_last = hosts_all[np.nonzero(in_window)[0]]
        sample = rng.choice(act_last, size=min(2048, len(act_last)), replace=False)
        log("timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(w, args.layout, slice0, sample, int(units), Lc)
        log("timing the CPU oracle on every host core")
        res["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w, args.layout, slice0, sample, int(units), Lc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
