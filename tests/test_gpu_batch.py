"""Batched steps (persistent work-queue kernels, graph replay) against the
same sketches stepped one by one through the single-sketch C ABI and against
the CPU oracle: BDR state bit-exact, estimates bit-exact (both sides form the
same exact integer sums and the same FP64 epilogue)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARAMS = [
    dict(m=70001, g=128, k=4, hash_seed=1, layout="fast"),
    dict(m=3 * 4096 + 17, g=256, k=16, hash_seed=2, layout="small"),
    dict(m=1 << 16, g=1024, k=128, hash_seed=3, layout="fast"),
    dict(m=20000, g=512, k=8, hash_seed=4, layout="small"),
    dict(m=(1 << 22) + 3, g=256, k=32, hash_seed=5, layout="fast"),
]


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_13132_amd import vbdr
    vbdr.lib()
    return vbdr


def _streams(seed, n_steps, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_steps):
        step = []
        for n in sizes:
            aips = rng.integers(0, 2**32, 200, dtype=np.uint64).astype(np.uint32)
            a = aips[rng.integers(0, 200, n)]
            b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32) % np.uint32(rng.integers(1000, 10**6))
            step.append(np.stack([a, b], 1).astype(np.uint32))
        out.append(step)
    return out


def _hosts(steps):
    return [np.unique(np.concatenate([st[i][:, 0] for st in steps] + [np.array([7, 8], np.uint32)]))
            for i in range(len(steps[0]))]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_single_sketches(V, use_graph):
    sizes = [5000, 0, 300000, 12345, 70000]  # uneven, one empty stream
    steps = _streams(1, 4, sizes)
    hosts = _hosts(steps)
    bt = V.Batch(PARAMS)
    bt.set_tuning(2048, 16, 4, use_graph)
    singles = [V.Sketch(p["m"], p["g"], p["k"], p["hash_seed"], p["layout"]) for p in PARAMS]
    hd = [V.to_device_u32(h) for h in hosts]
    for t, step in enumerate(steps):
        pd = [V.to_device_u32(p.reshape(-1)) for p in step]
        outs = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
        bt.step(pd, hd, outs)
        # eager work between replays on the caller's stream
        scratch = torch.ones(1 << 20, device="cuda").sum()
        for i, sk in enumerate(singles):
            sk.scan_slice(pd[i])
            sk.advance_slice()
        for i, sk in enumerate(singles):
            ref = sk.estimate(hd[i])
            assert torch.equal(outs[i], ref), f"step {t} sketch {i} estimates differ"
        assert float(scratch) == float(1 << 20)
    for i, (b, s) in enumerate(zip(bt.sketches, singles)):
        sb, ss = b.state(), s.state()
        for key in ("dr", "bs", "reg", "hist"):
            assert np.array_equal(sb[key], ss[key]), (i, key)
        assert sb["t"] == ss["t"] == len(steps)


def test_batch_matches_oracle(V):
    from oracle import oracle as O
    params = PARAMS
    sizes = [4000, 900, 20000, 3000, 50000]
    steps = _streams(2, 3, sizes)
    hosts = _hosts(steps)
    bt = V.Batch(params)
    # the member with 2^22 + 3 BDRs writes record runs and applies them in its advance
    assert [sk.info().scan_deferred for sk in bt.sketches] == [0, 0, 0, 0, 1]
    osks = [O.Sketch(p["m"], p["g"], p["k"], p["hash_seed"], O.GFAST if p["layout"] == "fast" else O.GSMALL)
            for p in params]
    hd = [V.to_device_u32(h) for h in hosts]
    for step in steps:
        outs = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
        bt.step([V.to_device_u32(p.reshape(-1)) for p in step], hd, outs)
        for i, osk in enumerate(osks):
            osk.scan(step[i])
            osk.advance()
            ref, raw = osk.estimate(hosts[i], with_raw=True)
            ref = ref.astype(np.float64)
            em = O.hll_from_hist(osk.state()["hist"], osk.m)
            floor = 1e-12 * (osk.m * np.abs(raw) + osk.g * em) / (osk.m - osk.g)
            got = outs[i].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref) + floor)
    for i, osk in enumerate(osks):
        sb, so = bt.sketches[i].state(), osk.state()
        for key in ("dr", "reg", "hist"):
            assert np.array_equal(sb[key], so[key]), (i, key)


def test_retuning_recaptures_and_autotuner(V):
    from paper_1810_13132_amd import autotune
    sizes = [20000, 5000, 60000, 1000, 8000]
    steps = _streams(3, 2, sizes)
    hosts = _hosts(steps)
    hd = [V.to_device_u32(h) for h in hosts]
    a, b = V.Batch(PARAMS), V.Batch(PARAMS)
    pd = [V.to_device_u32(p.reshape(-1)) for p in steps[0]]
    outs_a = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
    outs_b = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
    a.set_tuning(32768, 256, 16, True)
    a.step(pd, hd, outs_a)
    b.set_tuning(2048, 16, 4, True)
    b.step(pd, hd, outs_b)
    for x, y in zip(outs_a, outs_b):
        assert torch.equal(x, y)
    best, timings = autotune.tune(a, pd, hd, outs_a, candidates=[(2048, 16, 4), (8192, 64, 8)], reps=1)
    assert len(timings) == 2 and best["scan_tile"] in (2048, 8192)
    assert a.get_tuning()["scan_tile"] == best["scan_tile"]


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_batch_deferred_member_overflow(V, layout):
    """A member with record runs gets more records than its runs hold (about
    2.1 per BDR in a slice of 9e6 pairs; runs hold 2): the rest is applied by
    the scan directly and the next advance reads every plane.  Against the
    oracle after every step, and against the same sketch stepped alone."""
    from oracle import oracle as O
    params = [dict(m=(1 << 22) + 3, g=256, k=3, hash_seed=9, layout=layout),
              dict(m=5000, g=64, k=2, hash_seed=10, layout="small")]
    rng = np.random.default_rng(11)
    aips = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    sizes = [[9_000_000, 1000], [30000, 0], [0, 500], [70000, 2000]]
    bt = V.Batch(params)
    single = V.Sketch(**params[0])
    osk = O.Sketch(params[0]["m"], params[0]["g"], params[0]["k"], 9, O.GFAST if layout == "fast" else O.GSMALL)
    hosts = [aips, aips[:100]]
    hd = [V.to_device_u32(h) for h in hosts]
    for sz in sizes:
        step = [np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
                for n in sz]
        pd = [V.to_device_u32(p.reshape(-1)) for p in step]
        outs = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
        bt.step(pd, hd, outs)
        single.scan_slice(pd[0])
        single.advance_slice()
        osk.scan(step[0])
        osk.advance()
        assert torch.equal(outs[0], single.estimate(hd[0]))
        sb, so = bt.sketches[0].state(), osk.state()
        for key in ("dr", "reg", "hist"):
            assert np.array_equal(sb[key], so[key]), key
        ss = single.state()
        for key in ("dr", "bs", "reg", "hist"):
            assert np.array_equal(sb[key], ss[key]), key


def test_batch_estimate_reads_high_registers(V):
    """The batch estimate gathers registers from their nibble copy, where 15
    stands for 15 and more and sends the gather to the byte array.  DRs are
    planted so that about a third of the registers come out 15 or more after
    the step's advance (the highest recent LBP1 of a BDR is its register):
    the batch must give the estimates of the same sketches stepped alone,
    which gather the bytes."""
    params = [dict(m=1 << 16, g=1024, k=8, hash_seed=11, layout="small"),
              dict(m=(1 << 22) + 3, g=256, k=8, hash_seed=12, layout="small")]
    rng = np.random.default_rng(13)
    bt = V.Batch(params)
    singles = [V.Sketch(**p) for p in params]
    for b, s in zip(bt.sketches, singles):
        st = s.state()
        m, L = st["dr"].shape
        top = rng.integers(1, 15, m)
        hi = rng.random(m) < 0.33
        top[hi] = rng.integers(15, L + 1, int(hi.sum()))
        dr = np.full((m, L), 255, np.uint8)
        dr[np.arange(m), top - 1] = rng.integers(0, 4, m).astype(np.uint8)  # set within the last 4 slices
        reg = np.zeros(m, np.uint8)
        st.update(dr=dr, reg=reg, hist=np.bincount(reg, minlength=len(st["hist"])).astype(np.uint64))
        b.load_state(st)
        s.load_state(st)
    hosts = [rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32) for _ in params]
    hd = [V.to_device_u32(h) for h in hosts]
    pd = [V.to_device_u32(np.zeros(0, np.uint32)) for _ in params]
    outs = [torch.empty(len(h), dtype=torch.float32, device="cuda") for h in hosts]
    bt.step(pd, hd, outs)
    for i, s in enumerate(singles):
        s.advance_slice()
        reg, _ = s.registers()
        assert 0.25 < float((reg >= 15).mean()) < 0.4, i
        assert np.array_equal(bt.sketches[i].registers()[0], reg), i
        assert torch.equal(outs[i], s.estimate(hd[i])), i


def test_batch_learned_members(V):
    """Members with a learned estimator (vbdr_batch_set_mlp) get the learned
    estimates of the same sketch stepped alone (bit for bit); the others keep
    their plain estimates; removing the model returns the member to plain."""
    rng = np.random.default_rng(21)
    params = [dict(m=70001, g=128, k=4, hash_seed=1, layout="fast"),
              dict(m=1 << 18, g=256, k=4, hash_seed=2, layout="small"),
              dict(m=(1 << 22) + 3, g=256, k=8, hash_seed=5, layout="fast")]
    w = rng.standard_normal(V.MLP_PARAMS).astype(np.float32) * 0.1
    mlp = V.MLP(w)  # no envelope: every host takes the network's estimate
    bt = V.Batch(params)
    bt.set_mlp(1, mlp)
    bt.set_mlp(2, mlp)
    singles = [V.Sketch(**p) for p in params]
    sizes = [20000, 60000, 90000]
    aips = [rng.integers(0, 2**32, 300, dtype=np.uint64).astype(np.uint32) for _ in params]
    hd = [V.to_device_u32(a) for a in aips]
    for t in range(5):
        if t == 4:
            bt.set_mlp(2, None)
        pd = [V.to_device_u32(np.stack([a[rng.integers(0, len(a), n)],
                                        rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1)
                              .astype(np.uint32).reshape(-1)) for a, n in zip(aips, sizes)]
        outs = [torch.empty(len(a), dtype=torch.float32, device="cuda") for a in aips]
        bt.step(pd, hd, outs)
        for i, sk in enumerate(singles):
            sk.scan_slice(pd[i])
            sk.advance_slice()
        assert torch.equal(outs[0], singles[0].estimate(hd[0]))
        assert torch.equal(outs[1], singles[1].estimate_learned(mlp, hd[1]))
        ref2 = singles[2].estimate(hd[2]) if t == 4 else singles[2].estimate_learned(mlp, hd[2])
        assert torch.equal(outs[2], ref2), t
        assert not torch.equal(outs[1], singles[1].estimate(hd[1]))
