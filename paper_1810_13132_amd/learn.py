"""Train and evaluate the learned estimator (GPU).

Samples are (features, ln(1 + n)) of every host after every slice once the
window is full, on streams of one workload shape: by default the tiny workload
(2^12 hosts, 2^20 pairs per slice, 12 slices, m = 2^18, g = 256, k = 4):
training seeds 0..99 (10^6 samples drawn from the 3,686,400), evaluation seeds
100..109.  With --workload mid: the mid workload (2^14 hosts, 2^22 pairs per
slice, 24 slices, m = 2^20, g = 512, k = 16), training seeds 0..39, the same
evaluation seeds.  Features come from the library's own scan / advance /
feature kernels; the truth is the exact distinct count of the window's pairs
(Definition 1), computed on the device with sort-unique.  Training runs the
library's float32 Adam kernels.

With --workload stress (m = 2^24, g = 2048): a stress window holds 10^10 and
more distinct pairs, too many to replay and count exactly per training
stream, so samples come from synthetic windows (stress_window): a window's
registers depend only on the set of distinct pairs in it, so that set goes in
as one slice, made of uniform background pairs and planted hosts whose
opposite hosts are distinct by construction (the truth is their number).
Training windows 0..31, evaluation windows 100..103; the stress benchmark
then applies the network to the real stress stream (its pool holds about
4.7·10^9 distinct pairs, inside the background range of the windows).

    python -m paper_1810_13132_amd.learn --out paper_1810_13132_amd/weights/mlp_tiny.npz
    python -m paper_1810_13132_amd.learn --workload mid --train-seeds 40 \
        --out paper_1810_13132_amd/weights/mlp_mid.npz
    python -m paper_1810_13132_amd.learn --workload stress --train-seeds 32 \
        --out paper_1810_13132_amd/weights/mlp_stress.npz
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from paper_1810_13132_amd import synth, vbdr

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(PKG, "weights", "mlp_tiny.npz")
MID_WEIGHTS = os.path.join(PKG, "weights", "mlp_mid.npz")
STRESS_WEIGHTS = os.path.join(PKG, "weights", "mlp_stress.npz")
WORKLOADS = {"tiny": synth.TINY, "mid": synth.MID, "stress": synth.STRESS}
WEIGHTS = {"tiny": DEFAULT_WEIGHTS, "mid": MID_WEIGHTS, "stress": STRESS_WEIGHTS}
# distinct background pairs of a synthetic stress window: log-uniform over this
# range, around the pool occupancy of the stress stream's full window
STRESS_BG = (2.5e9, 9e9)
# above this plain estimate the stress network keeps the plain one.  The
# sharing noise of the plain estimate is about the HyperLogLog error of a
# host's g registers, each shared with E_m / m ~ 280 window pairs: 1.04 /
# sqrt(g) x g x 280 ~ 1.3e4; 10^5 is ~7.5 of those, so a small host's plain
# estimate stays below it, while a count above it is large against the noise
# (the plain estimate's relative error is a few per cent there, which a
# network trained on log counts does not reach)
STRESS_PLAIN_ABOVE = 1e5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def window_truth(window_keys, host_keys):
    """Exact |OP(aip)| over the window for each host (int64 aip keys)."""
    u = torch.unique(torch.cat(window_keys))
    # keys are aip << 32 | bip in int64: shift logically (mask the sign extension)
    vals, cnts = torch.unique((u >> 32) & 0xFFFFFFFF, return_counts=True)
    pos = torch.searchsorted(vals, host_keys).clamp(max=max(len(vals) - 1, 0))
    hit = vals[pos] == host_keys
    return torch.where(hit, cnts[pos], torch.zeros_like(cnts[pos]))


def stream_samples(seed: int, w=synth.TINY, layout="fast", mlp=None):
    """Per full window: features, truth, plain (and learned) estimates of all hosts."""
    st = synth.Stream(w.scaled(seed=seed))
    sk = vbdr.Sketch(w.m, w.g, w.k, seed, layout)
    hosts = vbdr.to_device_u32(st.aip)
    host_keys = torch.from_numpy(st.aip.astype(np.int64)).cuda()
    window, out = [], []
    for t in range(w.slices):
        pd = vbdr.to_device_u32(st.slice(t).reshape(-1))
        sk.scan_slice(pd)
        sk.advance_slice()
        p = pd.view(-1, 2).to(torch.int64) & 0xFFFFFFFF
        window.append((p[:, 0] << 32) | p[:, 1])
        window = window[-w.k:]
        if t >= w.k - 1:
            rec = {"feats": sk.features(hosts), "truth": window_truth(window, host_keys),
                   "plain": sk.estimate(hosts)}
            if mlp is not None:
                rec["learned"], rec["fallback"] = sk.estimate_learned(mlp, hosts, with_fallback=True)
            out.append(rec)
    sk.close()
    return out


def _as_i32(x: torch.Tensor) -> torch.Tensor:
    """int64 values 0..2^32-1 as the int32 with the same 32 bits."""
    return (((x + (1 << 31)) & 0xFFFFFFFF) - (1 << 31)).to(torch.int32)


def _bijection32(x: torch.Tensor, key: int) -> torch.Tensor:
    """A keyed bijection of 32-bit values held in int64 (odd multiplies and
    xor-shifts, the constants of Wellons' lowbias32): distinct inputs give
    distinct outputs.  Input generation only, not the estimator's hash."""
    M = 0xFFFFFFFF
    x = (x * 0x9E3779B1 + key) & M
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & M
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & M
    return x ^ (x >> 16)


def stress_window(seed: int, w=synth.STRESS, layout="small", mlp=None, n_small=1 << 14, n_large=768,
                  n_bg=None):
    """One synthetic window of the stress shape (m, g of `w`): its distinct
    pairs scanned as one slice of a k = 1 sketch, then closed.  Background:
    n_bg uniform random pairs (aip below 2^31; log-uniform in STRESS_BG by
    default).  Planted hosts (aip 2^31 and above, distinct): n_small with
    Zipf(1.5) on 1..10^4 opposite hosts like the stream's background hosts and
    n_large log-uniform on 10^4..10^7 like its superspreaders, the opposite
    hosts of each distinct (a keyed bijection of 0..n-1).  Returns features,
    truth (the planted counts), plain (and learned) estimates of the planted
    hosts, and the background size."""
    rng = np.random.default_rng(7919 + seed)
    if n_bg is None:
        n_bg = int(math.exp(rng.uniform(math.log(STRESS_BG[0]), math.log(STRESS_BG[1]))))
    sk = vbdr.Sketch(w.m, w.g, 1, seed, layout)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(104729 + seed)
    done, chunk = 0, 1 << 26
    while done < n_bg:
        c = min(chunk, n_bg - done)
        pd = torch.randint(0, 1 << 32, (c, 2), dtype=torch.int64, device="cuda", generator=gen)
        pd[:, 0] &= 0x7FFFFFFF
        sk.scan_slice(_as_i32(pd).view(-1))
        done += c
        del pd
    ks = np.arange(1, 10**4 + 1, dtype=np.float64)
    cdf = np.cumsum(ks ** -1.5)
    small = 1 + np.searchsorted(cdf / cdf[-1], rng.random(n_small))
    large = np.exp(rng.uniform(math.log(1e4), math.log(1e7), n_large)).astype(np.int64)
    counts = np.concatenate([small, large]).astype(np.int64)
    addr = np.unique(rng.integers(0, 1 << 31, 2 * len(counts), dtype=np.int64))
    addr = rng.permutation(addr)[:len(counts)] | (1 << 31)
    keys = rng.integers(0, 1 << 32, len(counts), dtype=np.int64)
    # the planted pairs, a block of hosts at a time (at most ~2^26 pairs)
    i = 0
    while i < len(counts):
        j, tot = i, 0
        while j < len(counts) and (tot == 0 or tot + counts[j] <= chunk):
            tot += int(counts[j])
            j += 1
        cnt = torch.from_numpy(counts[i:j]).cuda()
        start = torch.cumsum(cnt, 0) - cnt
        host = torch.repeat_interleave(torch.arange(j - i, device="cuda"), cnt)
        local = torch.arange(tot, device="cuda") - start[host]
        bip = _bijection32(local, 0) ^ torch.from_numpy(keys[i:j]).cuda()[host]
        aip = torch.from_numpy(addr[i:j]).cuda()[host]
        sk.scan_slice(_as_i32(torch.stack([aip, bip], 1)).view(-1))
        i = j
    sk.advance_slice()
    hosts = vbdr.to_device_u32(addr.astype(np.uint32))
    rec = {"feats": sk.features(hosts), "truth": torch.from_numpy(counts).cuda(), "plain": sk.estimate(hosts),
           "n_bg": n_bg, "n_large": n_large}
    if mlp is not None:
        rec["learned"], rec["fallback"] = sk.estimate_learned(mlp, hosts, with_fallback=True)
    sk.close()
    return rec


def window_samples(seed: int, w, mlp=None):
    """The samples of one training or evaluation seed of workload `w`."""
    if w.name == "stress":
        return [stress_window(seed, w, mlp=mlp)]
    return stream_samples(seed, w, mlp=mlp)


def rms_rel(est, truth):
    t = truth.to(torch.float64)
    keep = t >= 1
    r = (est.to(torch.float64)[keep] - t[keep]) / t[keep]
    return float(torch.sqrt(torch.mean(r * r)))


def envelope(feats: torch.Tensor):
    lo = feats.min(0).values.double()
    hi = feats.max(0).values.double()
    span = hi - lo
    pad = torch.maximum(0.05 * span, 1e-3 * torch.maximum(lo.abs(), hi.abs()) + 1e-6)
    return (lo - pad).float().cpu().numpy(), (hi + pad).float().cpu().numpy()


def init_params(seed: int):
    """He-uniform init; output bias at the mean target."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan in (((64, 67), 67), ((64,), None), ((64, 64), 64), ((64,), None), ((64,), 64), ((1,), None)):
        n = int(np.prod(shape))
        parts.append(rng.uniform(-math.sqrt(6 / fan), math.sqrt(6 / fan), n) if fan else np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def train(train_seeds=range(100), n_samples=10**6, epochs=30, batch=4096, lr=3e-3, seed=0, w=synth.TINY):
    t0 = time.time()
    feats, targets = [], []
    for s in train_seeds:
        for rec in window_samples(s, w):
            feats.append(rec["feats"])
            targets.append(torch.log1p(rec["truth"].to(torch.float32)))
        if s % 10 == 9 or w.name == "stress":
            log(f"train seed {s}: {sum(len(t) for t in targets)} samples ({time.time() - t0:.1f}s)")
    X = torch.cat(feats)
    Y = torch.cat(targets)
    g = torch.Generator(device="cpu").manual_seed(seed)
    pick = torch.randperm(len(Y), generator=g)[:n_samples].cuda()
    X, Y = X[pick].contiguous(), Y[pick].contiguous()
    lo, hi = envelope(X)
    params = init_params(seed)
    params[-1] = float(Y.mean())
    tr = vbdr.Trainer(params, lr)
    steps_per_epoch = len(Y) // batch
    total = epochs * steps_per_epoch
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(len(Y), generator=g).cuda()
        loss.zero_()
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            tr.set_lr(lr * 0.5 * (1 + math.cos(math.pi * step / total)) + 1e-5)
            tr.step(X[idx].contiguous(), Y[idx].contiguous(), loss)
            step += 1
        log(f"epoch {ep}: mean batch loss {float(loss.cpu()[0]) / steps_per_epoch:.5f} ({time.time() - t0:.1f}s)")
    return tr.params(), lo, hi, {"samples": int(len(Y)), "epochs": epochs, "batch": batch, "lr": lr,
                                 "train_seeds": [min(train_seeds), max(train_seeds)], "workload": w.name}


def evaluate(params, lo, hi, eval_seeds=range(100, 110), w=synth.TINY, plain_above=None):
    mlp = vbdr.MLP(params, lo, hi, plain_above)
    ests, truths, plains, fbs = [], [], [], []
    for s in eval_seeds:
        for rec in window_samples(s, w, mlp=mlp):
            ests.append(rec["learned"])
            plains.append(rec["plain"])
            truths.append(rec["truth"])
            fbs.append(rec["fallback"])
    est, plain, truth, fb = torch.cat(ests), torch.cat(plains), torch.cat(truths), torch.cat(fbs)
    res = {"samples": int(len(truth)), "samples_n_ge_1": int((truth >= 1).sum()),
           "rms_rel_plain": rms_rel(plain, truth), "rms_rel_learned": rms_rel(est, truth),
           "fallback_frac": float((fb == 1).float().mean()), "eval_seeds": [min(eval_seeds), max(eval_seeds)]}
    if w.name == "stress":  # the planted heavy hosts apart (10^4..10^7), as the stress benchmark reports them
        res["kept_plain_frac"] = float((fb == 2).float().mean())
        big = truth >= 10**4
        res["rms_rel_plain_large"] = rms_rel(plain[big], truth[big])
        res["rms_rel_learned_large"] = rms_rel(est[big], truth[big])
        res["rms_rel_plain_small"] = rms_rel(plain[~big], truth[~big])
        res["rms_rel_learned_small"] = rms_rel(est[~big], truth[~big])
        return res
    # estimation throughput on the same sketch shape with a full window, the
    # stream's hosts repeated to 2^18 estimates per launch, plain vs learned
    st = synth.Stream(w.scaled(seed=min(eval_seeds)))
    sk = vbdr.Sketch(w.m, w.g, w.k, 0, "fast")
    for t in range(w.k):
        sk.scan_slice(vbdr.to_device_u32(st.slice(t).reshape(-1)))
        sk.advance_slice()
    hosts = vbdr.to_device_u32(np.tile(st.aip, max(1, (1 << 18) // w.hosts)))
    out = torch.empty(hosts.numel(), dtype=torch.float32, device="cuda")

    def rate(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            fn()
        b.record()
        b.synchronize()
        return hosts.numel() * 10 / (a.elapsed_time(b) * 1e-3)

    res["hosts_per_s_plain"] = rate(lambda: sk.estimate(hosts, out))
    res["hosts_per_s_learned"] = rate(lambda: sk.estimate_learned(mlp, hosts, out))
    return res


def load(path=DEFAULT_WEIGHTS):
    z = np.load(path, allow_pickle=False)
    return z["params"], z["env_lo"], z["env_hi"], json.loads(str(z["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="tiny", choices=sorted(WORKLOADS))
    ap.add_argument("--out", default=None)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--train-seeds", type=int, default=100)
    ap.add_argument("--samples", type=int, default=10**6)
    ap.add_argument("--eval-only", action="store_true")
    args = ap.parse_args()
    w = WORKLOADS[args.workload]
    if args.out is None:
        args.out = WEIGHTS[args.workload]
    if args.eval_only:
        params, lo, hi, meta = load(args.out)
        if w.name == "stress":
            meta["plain_above"] = STRESS_PLAIN_ABOVE
    else:
        params, lo, hi, meta = train(range(args.train_seeds), args.samples, args.epochs, w=w)
        if w.name == "stress":
            meta["plain_above"] = STRESS_PLAIN_ABOVE
    res = evaluate(params, lo, hi, eval_seeds=range(100, 104) if w.name == "stress" else range(100, 110), w=w,
                   plain_above=meta.get("plain_above"))
    meta["eval"] = res
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, params=params, env_lo=lo, env_hi=hi, meta=np.array(json.dumps(meta)))
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
