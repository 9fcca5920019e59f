"""HIP path vs CPU oracle, element by element, through the C ABI.

BDR state (every DR, the open slice's bsLBP1, every register, the pool
histogram) must match bit for bit after every scan and every advance;
register histograms per host bit for bit; FP32 estimates within 1e-6
relative of the FP64 oracle, plus an absolute floor for the cancellation in
(m E_s - g E_m) / (m - g): the two sides run the same FP64 operations in the
same order and differ only in the last bit of log(), so the floor is a few
FP64 ulps of the cancelled terms.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

LAYOUT_CODE = {"fast": 1, "small": 2}  # oracle layout codes


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_13132_amd import vbdr
    vbdr.lib()
    return vbdr


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _dev(V, a):
    return V.to_device_u32(a)


def _random_slices(seed, n_slices, max_pairs, n_aip, n_bip, empty_prob=0.1):
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, n_aip, dtype=np.uint64).astype(np.uint32)
    bips = rng.integers(0, 2**32, n_bip, dtype=np.uint64).astype(np.uint32)
    out = []
    for _ in range(n_slices):
        n = 0 if rng.random() < empty_prob else int(rng.integers(1, max_pairs + 1))
        out.append(np.stack([aips[rng.integers(0, n_aip, n)], bips[rng.integers(0, n_bip, n)]], 1)
                   .astype(np.uint32).reshape(-1, 2))
    return aips, out


def assert_state_equal(gs, os_, layout, where):
    assert gs["t"] == os_["t"], where
    assert np.array_equal(gs["dr"], os_["dr"]), f"DR mismatch {where}: {np.argwhere(gs['dr'] != os_['dr'])[:5]}"
    if layout == "fast":
        assert np.array_equal(gs["bs"], os_["bs"]), f"bsLBP1 mismatch {where}"
    else:
        assert not gs["bs"].any()
    assert np.array_equal(gs["reg"], os_["reg"]), f"register mismatch {where}"
    assert np.array_equal(gs["hist"], os_["hist"]), f"pool histogram mismatch {where}"


def assert_estimates_close(V, O, sk, osk, hosts):
    hd = _dev(V, hosts)
    out, raw, hist = sk.estimate_ex(hd)
    plain = sk.estimate(hd)
    torch.cuda.synchronize()
    out, raw, hist, plain = out.cpu().numpy(), raw.cpu().numpy(), hist.cpu().numpy(), plain.cpu().numpy()
    ref, ref_raw, ref_hist = osk.estimate(hosts, with_raw=True, with_hist=True)
    assert np.array_equal(hist.astype(np.uint32), ref_hist), "per-host register histogram mismatch"
    assert np.array_equal(out, plain), "estimate and estimate_ex disagree"
    np.testing.assert_allclose(raw, ref_raw, rtol=1e-13, atol=0)
    em = O.hll_from_hist(osk.state()["hist"], osk.m)
    m, g = float(osk.m), float(osk.g)
    floor = 1e-12 * (m * np.abs(ref_raw) + g * em) / (m - g)
    err = np.abs(out.astype(np.float64) - ref.astype(np.float64))
    bad = err > 1e-6 * np.abs(ref.astype(np.float64)) + floor
    assert not bad.any(), f"estimates off at {np.nonzero(bad)[0][:5]}: gpu {out[bad][:5]} ref {ref[bad][:5]}"
    return ref


def run_parity(V, O, layout, m, g, k, seed, slices, hosts, split=1):
    sk = V.Sketch(m, g, k, seed, layout)
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE[layout])
    for t, pairs in enumerate(slices):
        pd = _dev(V, pairs.reshape(-1))
        n = len(pairs)
        cuts = np.linspace(0, n, split + 1).astype(int)
        for a, b in zip(cuts[:-1], cuts[1:]):
            sk.scan_slice(pd[2 * a: 2 * b])
        osk.scan(pairs)
        assert_state_equal(sk.state(), osk.state(), layout, f"after scan of slice {t}")
        sk.advance_slice()
        osk.advance()
        assert_state_equal(sk.state(), osk.state(), layout, f"after advance of slice {t}")
        if len(hosts):
            assert_estimates_close(V, O, sk, osk, hosts)
    return sk, osk


@pytest.mark.parametrize("layout", ["fast", "small"])
@pytest.mark.parametrize("m,g,k,seed", [
    (3 * 4096 + 123, 64, 3, 1),      # ragged pool, several advance tiles
    (5000, 2, 1, 2),                 # b = 1: L = 32, discrete window
    (70001, 65536, 7, 3),            # g above the LDS-staged seed table
    (4097, 16, 254, 4),              # largest window
])
def test_parity_random_streams(V, O, layout, m, g, k, seed):
    aips, slices = _random_slices(seed, 9, 6000, 40, 3000)
    hosts = np.concatenate([aips[:33], np.array([12345, 0, 0xFFFFFFFF], np.uint32)])
    run_parity(V, O, layout, m, g, k, seed, slices, hosts, split=3)


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_parity_saturation_long_history(V, O, layout):
    """300 slices: DRs climb to 255 and stay (no wrap)."""
    aips, slices = _random_slices(7, 300, 20, 3, 50, empty_prob=0.8)
    sk = V.Sketch(4096 + 5, 8, 5, 9, layout)
    osk = O.Sketch(4096 + 5, 8, 5, 9, LAYOUT_CODE[layout])
    for pairs in slices:
        if len(pairs):
            sk.scan_slice(_dev(V, pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
    gs, os_ = sk.state(), osk.state()
    assert_state_equal(gs, os_, layout, "after 300 slices")
    assert (gs["dr"] == 255).any()
    assert_estimates_close(V, O, sk, osk, aips)


def test_empty_inputs(V, O):
    sk = V.Sketch(10000, 32, 3, 5, "fast")
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    sk.scan_slice(empty)
    out = sk.estimate(empty)
    assert out.numel() == 0
    hosts = _dev(V, np.arange(100, dtype=np.uint32))
    assert not sk.estimate(hosts).cpu().numpy().any()  # before any advance
    sk.advance_slice()
    sk.advance_slice()
    assert not sk.estimate(hosts).cpu().numpy().any()
    s = sk.state()
    assert s["t"] == 2 and s["hist"][0] == 10000 and (s["dr"] == 255).all() and not s["reg"].any()


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_parity_tiny_workload(V, O, layout):
    """The tiny workload at its full size: 2^12 hosts, 2^20 pairs per slice,
    12 slices, m = 2^18, g = 256, k = 4; every host estimated each slice."""
    from paper_1810_13132_amd import synth
    w = synth.TINY
    st = synth.Stream(w)
    sk = V.Sketch(w.m, w.g, w.k, w.seed, layout)
    osk = O.Sketch(w.m, w.g, w.k, w.seed, LAYOUT_CODE[layout])
    hosts = st.aip
    for t in range(w.slices):
        pairs = st.slice(t)
        sk.scan_slice(_dev(V, pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
        if t in (0, 3, w.slices - 1):
            assert_state_equal(sk.state(), osk.state(), layout, f"slice {t}")
        assert_estimates_close(V, O, sk, osk, hosts)


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_parity_large_pool_partitioned_estimate(V, O, layout):
    """Pools of 2^22 BDRs and more take the XCD-partitioned estimate (default
    below 2^24 BDRs) or the LDS-tiled one; more hosts than one pass or block
    holds (2^17) exercise the chunking.  The plain estimate is checked against
    the oracle and against estimate_ex (direct gathers), and every variant must
    agree with it bit for bit."""
    m, g, k, seed = (1 << 22) + 77, 256, 3, 13
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, 5000, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, layout)
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE[layout])
    for t in range(3):
        n = 1 << 19
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        sk.scan_slice(_dev(V, pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
    assert_state_equal(sk.state(), osk.state(), layout, "large pool")
    hosts = np.concatenate([aips, rng.integers(0, 2**32, (1 << 17) + 3000 - len(aips), dtype=np.uint64)
                            .astype(np.uint32)])
    ref = assert_estimates_close(V, O, sk, osk, hosts)
    assert (ref[: len(aips)] > 0).all()
    # resume: the imported registers must feed the partitioned path too
    b = V.Sketch(m, g, k, seed, layout)
    b.load_state(sk.state())
    hd = _dev(V, hosts)
    plain = sk.estimate(hd)
    assert torch.equal(b.estimate(hd), plain)
    # below 2^24 BDRs the default is the XCD-partitioned estimate
    assert sk.info().est_tiled == 0 and sk.info().est_parts == 8
    # the binned estimate (each (host, i) hashed once) gives the same bits,
    # in one pass, in ragged passes, and with runs too short for most hosts
    for tune in ({}, {"est_bin_hosts": 40000}, {"est_bin_cap": 20}, {"est_bin_hosts": 999, "est_bin_cap": 33}):
        sk.set_tuning(est_binned=1, **tune)
        assert torch.equal(sk.estimate(hd), plain), tune
    # the LDS-tiled estimate: one block; buckets and runs too short for most tiles
    # (their overflow is gathered directly); 33 blocks of at most 4096 hosts
    for tune in ({}, {"est_bin_cap": 40}, {"est_bin_cap": 9}, {"est_bin_hosts": 5000}):
        sk.set_tuning(est_binned=3, **tune)
        assert torch.equal(sk.estimate(hd), plain), tune


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_binned_estimate_pow2_pool_ragged_g(V, O, layout):
    """A power-of-two pool takes the shift form of H(x, m, A) in the binned
    estimate; g = 128 fills only half a row of hashes per host.  Both
    estimate variants against the oracle."""
    m, g, k, seed = 1 << 22, 128, 2, 21
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, layout)
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE[layout])
    for t in range(2):
        n = 1 << 18
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        sk.scan_slice(_dev(V, pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
    hosts = np.concatenate([aips, rng.integers(0, 2**32, 2001, dtype=np.uint64).astype(np.uint32)])
    assert_estimates_close(V, O, sk, osk, hosts)
    hd = _dev(V, hosts)
    plain = sk.estimate(hd)
    for tune in ({"est_binned": 2}, {"est_binned": 1}, {"est_binned": 1, "est_bin_cap": 10}, {"est_binned": 3},
                 {"est_binned": 3, "est_bin_cap": 7}):
        sk.set_tuning(**tune)
        assert torch.equal(sk.estimate(hd), plain), tune


def test_two_stream_schedule_matches_one_stream(V):
    """Slice t+1's scan may run on a second stream while slice t is estimated
    (it needs only slice t's advance).  That schedule gives the same estimates
    and the same state as the sequential one, with deferred scans and the
    tiled estimate."""
    m, g, k = 1 << 22, 256, 3
    rng = np.random.default_rng(17)
    aips = rng.integers(0, 2**32, 4000, dtype=np.uint64).astype(np.uint32)
    hd = _dev(V, aips)
    a = V.Sketch(m, g, k, 5, "small")
    b = V.Sketch(m, g, k, 5, "small")
    for s_ in (a, b):
        s_.set_tuning(est_binned=3)
    assert a.info().est_tiled == 1 and a.info().scan_deferred == 1
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()
    slices = []
    for t in range(5):
        n = 1 << 19
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        slices.append(_dev(V, pairs.reshape(-1)))
    outs_a, outs_b, adv = [], [], None
    for t in range(5):
        a.scan_slice(slices[t])
        a.advance_slice()
        outs_a.append(a.estimate(hd))
        if adv is not None:
            side.wait_event(adv)
        b.scan_slice(slices[t], stream=side)
        done = torch.cuda.Event()
        done.record(side)
        main.wait_event(done)
        b.advance_slice(stream=main)
        adv = torch.cuda.Event()
        adv.record(main)
        outs_b.append(b.estimate(hd, stream=main))
    torch.cuda.synchronize()
    for t in range(5):
        assert torch.equal(outs_a[t], outs_b[t]), t
    sa, sb = a.state(), b.state()
    for key in ("dr", "reg", "hist"):
        assert np.array_equal(sa[key], sb[key]), key


@pytest.mark.parametrize("g,m", [(64, 1 << 22), (2048, (1 << 22) + 12345), (8192, 1 << 22), (1024, (1 << 23) + 3)])
def test_tiled_estimate_edge_g(V, O, g, m):
    """The tiled estimate at the ends of its g range: g = 64 (chunks of 64
    hosts, half a chunk of pairs per thread unused), g = 2048 and 8192 (one
    host spans several pair slots of every thread), on power-of-two pools
    (the pool index a shift of the hash) and others (a high multiply).
    Bit-identical to the partitioned and the direct gathers, and within the
    bar of the oracle."""
    k, seed = 2, 3
    rng = np.random.default_rng(g)
    aips = rng.integers(0, 2**32, 1500, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, "small")
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE["small"])
    for t in range(2):
        n = 1 << 18
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        sk.scan_slice(_dev(V, pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
    hosts = np.concatenate([aips, rng.integers(0, 2**32, 2049, dtype=np.uint64).astype(np.uint32)])
    assert_estimates_close(V, O, sk, osk, hosts)
    hd = _dev(V, hosts)
    direct = sk.estimate_ex(hd)[0]
    sk.set_tuning(est_binned=3)
    assert sk.info().est_tiled == 1
    tiled = sk.estimate(hd)
    sk.set_tuning(est_binned=3, est_bin_hosts=2048)  # two blocks, the second ragged
    tiled2 = sk.estimate(hd)
    sk.set_tuning(est_binned=2)
    part = sk.estimate(hd)
    assert torch.equal(tiled, direct) and torch.equal(tiled2, direct) and torch.equal(part, direct)


@pytest.mark.parametrize("g,lo", [(256, 0), (8192, 3), (1024, 3)])
def test_tiled_estimate_high_registers(V, O, g, lo):
    """Registers of 15 and more do not fit the tiled estimate's nibble tile:
    they are listed and read from the byte array.  Registers lo..L are planted
    through import (a third of them 15 or more); each sampled host's register
    histogram must be the one the oracle's getPhyIdx (Alg. 3) gives over the
    planted registers, its raw E_s the oracle's HyperLogLog of that histogram,
    and every estimate path must give the same bits.  With lo = 3 and 0.5 % of
    the registers set to 0, 1 or 2 the tiled estimate keeps 16-bit per-tile
    sums (registers 0..2 below 1/64 of the pool) carrying zero counts; at g =
    8192 (about 32 records of a host per tile) most of them exceed 16 bits and
    go to the host's overflow sum."""
    m, k, seed = 1 << 22, 3, 29
    rng = np.random.default_rng(29 + g)
    a = V.Sketch(m, g, k, seed, "small")
    st = a.state()
    reg = rng.integers(lo, 15, m).astype(np.uint8)
    if lo:
        low = rng.random(m) < 0.005
        reg[low] = rng.integers(0, lo, int(low.sum())).astype(np.uint8)
    hi = rng.random(m) < 0.33
    reg[hi] = rng.integers(15, a.L + 1, int(hi.sum())).astype(np.uint8)
    st["reg"], st["hist"] = reg, np.bincount(reg, minlength=len(st["hist"])).astype(np.uint64)
    b = V.Sketch(m, g, k, seed, "small")
    b.load_state(st)
    hosts = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    hd = _dev(V, hosts)
    out, raw, hh = b.estimate_ex(hd)
    raw, hh = raw.cpu().numpy(), hh.cpu().numpy()
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE["small"])
    for j in range(0, len(hosts), 97 if g <= 1024 else 499):
        idx = [osk.phy_idx(int(hosts[j]), i) for i in range(g)]
        want = np.bincount(reg[idx], minlength=hh.shape[1])
        assert np.array_equal(hh[j], want), j
        assert (reg[idx] >= 15).any(), j
        np.testing.assert_allclose(raw[j], O.hll_from_hist(want, g), rtol=1e-13, atol=0)
    for tune in ({"est_binned": 3}, {"est_binned": 3, "est_bin_cap": 40}, {"est_binned": 3, "est_bin_hosts": 2048},
                 {"est_binned": 2}, {"est_binned": 1}):
        b.set_tuning(**tune)
        if tune["est_binned"] == 3:
            assert b.info().est_tiled == 1
        assert torch.equal(b.estimate(hd), out), tune


def test_tiled_workspace_follows_block_size(V):
    """est_bin_hosts sizes the tiled estimate's workspace: a smaller block
    frees most of it, the estimates stay bit for bit the same, and the
    default tuning brings the full workspace back."""
    m, g, k = 1 << 24, 1024, 4
    sk = V.Sketch(m, g, k, 3, "small")
    rng = np.random.default_rng(11)
    aips = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    for _ in range(3):
        n = 1 << 20
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        sk.scan_slice(V.to_device_u32(pairs.reshape(-1)))
        sk.advance_slice()
    hosts = _dev(V, np.concatenate([aips, rng.integers(0, 2**32, 9000, dtype=np.uint64).astype(np.uint32)]))
    full = sk.info().workspace_bytes
    ref = sk.estimate(hosts)
    sk.set_tuning(est_binned=3, est_bin_hosts=4096)
    small = sk.info().workspace_bytes
    assert small < full / 4, (small, full)
    assert torch.equal(sk.estimate(hosts), ref)
    sk.set_tuning()
    assert sk.info().workspace_bytes == full
    assert torch.equal(sk.estimate(hosts), ref)


def test_default_estimate_by_pool_size(V):
    """Pools from 2^24 BDRs default to the LDS-tiled estimate, smaller ones to
    the partitioned one; on the same sketch the tiled, partitioned and direct
    (estimate_ex) gathers agree bit for bit."""
    assert V.Sketch((1 << 24) - 4096, 1024, 4, 3, "small").info().est_tiled == 0
    m, g, k = 1 << 24, 1024, 4
    sk = V.Sketch(m, g, k, 3, "small")
    assert sk.info().est_tiled == 1
    rng = np.random.default_rng(3)
    aips = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    for t in range(2):
        n = 1 << 20
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        sk.scan_slice(_dev(V, pairs.reshape(-1)))
        sk.advance_slice()
    hosts = np.concatenate([aips, rng.integers(0, 2**32, 1001, dtype=np.uint64).astype(np.uint32)])
    hd = _dev(V, hosts)
    tiled = sk.estimate(hd)
    direct = sk.estimate_ex(hd)[0]
    sk.set_tuning(est_binned=2)
    assert sk.info().est_tiled == 0
    part = sk.estimate(hd)
    assert torch.equal(tiled, part) and torch.equal(tiled, direct)
    assert (tiled[: len(aips)] > 0).all()


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_binned_scan_matches_direct_and_overflows_safely(V, O, layout):
    """Large pools scan in two passes through per-XCD bins.  A slice of one
    repeated pair plus noise sends more records to one bin than it holds
    (2^21 + 2^19 + 2^16 per 2^24-pair pass), exercising the direct fallback."""
    m, g, k, seed = (1 << 22) + 5, 256, 5, 17
    rng = np.random.default_rng(seed)
    n_rep, n_rand = 3 << 20, 1 << 18
    rep = np.tile(np.array([[123456789, 987654321]], np.uint32), (n_rep, 1))
    rnd = rng.integers(0, 2**32, (n_rand, 2), dtype=np.uint64).astype(np.uint32)
    slices = [np.concatenate([rep, rnd])[rng.permutation(n_rep + n_rand)], rnd[::-1].copy()]
    a = V.Sketch(m, g, k, seed, layout)
    a.set_tuning(scan_binned=1, scan_defer=2)  # binned
    b = V.Sketch(m, g, k, seed, layout)
    b.set_tuning(scan_binned=2, scan_defer=2)  # direct
    c = V.Sketch(m, g, k, seed, layout)  # deferred (default): one tile's run overflows into direct updates
    assert a.get_tuning()["scan_binned"] == 1 and c.info().scan_deferred == 1 and b.info().scan_deferred == 0
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE[layout])
    for pairs in slices:
        pd = _dev(V, pairs.reshape(-1))
        a.scan_slice(pd)
        b.scan_slice(pd)
        c.scan_slice(pd)
        osk.scan(pairs)
        sa, sb, sc = a.state(), b.state(), c.state()
        assert_state_equal(sa, osk.state(), layout, "binned scan vs oracle (open slice)")
        for key in ("dr", "bs", "reg", "hist"):
            assert np.array_equal(sa[key], sb[key]), key
            assert np.array_equal(sc[key], sb[key]), key
        a.advance_slice()
        b.advance_slice()
        c.advance_slice()
        osk.advance()
    assert_state_equal(a.state(), osk.state(), layout, "binned scan vs oracle (closed)")
    assert_state_equal(c.state(), osk.state(), layout, "deferred scan vs oracle (closed)")


@pytest.mark.parametrize("layout", ["fast", "small"])
def test_deferred_scan_parity(V, O, layout):
    """Large pools defer the scan's updates to the advance (records sorted by
    tile of 2^15 BDRs).  A ragged pool (last tile partial), several scan
    calls per slice, a state export in the middle of a slice (pending records
    applied first), an empty slice, and switches of the mode in the middle of
    a slice; the state after every advance and the estimates against the
    oracle."""
    m, g, k, seed = (1 << 22) + 77, 512, 3, 23
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, 4000, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, layout)
    assert sk.get_tuning()["scan_defer"] == 1 and sk.info().scan_deferred == 1
    osk = O.Sketch(m, g, k, seed, LAYOUT_CODE[layout])
    hosts = aips[:700]
    for t in range(6):
        n = 0 if t == 3 else int(rng.integers(1 << 18, 1 << 19))
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        pd = _dev(V, pairs.reshape(-1))
        cuts = [0, n // 3, n // 2, n]
        for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
            if t == 4 and i == 1:
                sk.set_tuning(scan_defer=2)  # pending records go to the pool
            if t == 5 and i == 1:
                sk.set_tuning(scan_defer=1)  # back, with bsLBP1 bits already set
            sk.scan_slice(pd[2 * a: 2 * b])
            if t == 1 and i == 0:
                osk.scan(pairs[:b])
                assert_state_equal(sk.state(), osk.state(), layout, "mid-slice export")
                osk.scan(pairs[b:])
        if t != 1:
            osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
        assert_state_equal(sk.state(), osk.state(), layout, f"after advance of slice {t}")
        assert_estimates_close(V, O, sk, osk, hosts)
    # resume in the middle of a slice: the export applies the pending records,
    # the import hands them to the next advance as pool state
    n = 1 << 18
    pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                      rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
    sk.scan_slice(_dev(V, pairs.reshape(-1)))
    mid = sk.state()
    b = V.Sketch(m, g, k, seed, layout)
    b.load_state(mid)
    sk.advance_slice()
    b.advance_slice()
    osk.scan(pairs)
    osk.advance()
    assert_state_equal(b.state(), osk.state(), layout, "resumed")
    assert_state_equal(sk.state(), osk.state(), layout, "continued")


def test_resume_from_exported_state(V, O):
    """Export after 5 slices, import into a fresh sketch, continue: identical
    to an uninterrupted run."""
    aips, slices = _random_slices(11, 10, 3000, 30, 2000)
    m, g, k = 9000, 32, 4
    a = V.Sketch(m, g, k, 21, "fast")
    for i, pairs in enumerate(slices):
        if len(pairs):
            a.scan_slice(_dev(V, pairs.reshape(-1)))
        if i == 5:
            mid = a.state()  # open slice with bsLBP1 bits set
        a.advance_slice()
    b = V.Sketch(m, g, k, 21, "fast")
    b.load_state(mid)
    assert_state_equal(b.state(), mid, "fast", "after import")
    b.advance_slice()
    for pairs in slices[6:]:
        if len(pairs):
            b.scan_slice(_dev(V, pairs.reshape(-1)))
        b.advance_slice()
    assert_state_equal(b.state(), a.state(), "fast", "resumed vs continuous")


@pytest.mark.parametrize("layout", ["fast", "small", "packed"])
def test_import_over_saturated_planes(V, O, layout):
    """The deferred advance skips planes it found saturated (all 255, or
    2^z - 1 for the packed layout) last time.  Importing a state into a sketch that has run (its masks say
    saturated where the imported DRs are not), flushing pending records on
    export, and overflowing record runs all change DRs outside the advance;
    each must make the next advance read every plane.  Checked against the
    oracle after every slice."""
    m, g, k = 1 << 22, 64, 3
    rng = np.random.default_rng(41)
    aips = rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)

    def slice_pairs(n):
        return np.stack([aips[rng.integers(0, len(aips), n)],
                         rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)

    Lc = 24 if layout == "packed" else 0  # L = 27 at g = 64: the top recorders merge
    a = V.Sketch(m, g, k, 9, layout, Lc=Lc)
    a.scan_slice(_dev(V, slice_pairs(1 << 16).reshape(-1)))
    a.advance_slice()  # most planes of most groups saturated
    src = V.Sketch(m, g, k, 9, layout, Lc=Lc)
    osk = O.Sketch(m, g, k, 9, O.GPACKED if layout == "packed" else LAYOUT_CODE[layout], Lc=Lc)
    for t in range(3):
        p_ = slice_pairs(1 << 19)
        src.scan_slice(_dev(V, p_.reshape(-1)))
        osk.scan(p_)
        src.advance_slice()
        osk.advance()
    a.load_state(src.state())
    assert a.info().scan_deferred == 1
    for t in range(3):
        p_ = slice_pairs(1 << 18)
        if t == 1:  # one BDR's pair repeated past its run: direct updates
            p_[: 1 << 17] = p_[0]
        a.scan_slice(_dev(V, p_[: len(p_) // 2].reshape(-1)))
        osk.scan(p_[: len(p_) // 2])
        if t == 2:  # export in mid-slice applies the pending records
            assert_state_equal(a.state(), osk.state(), layout, "mid-slice")
        a.scan_slice(_dev(V, p_[len(p_) // 2:].reshape(-1)))
        osk.scan(p_[len(p_) // 2:])
        a.advance_slice()
        osk.advance()
        assert_state_equal(a.state(), osk.state(), layout, f"slice {t} after import")


def test_bad_arguments_on_device(V):
    sk = V.Sketch(5000, 16, 3, 1, "small")
    pairs = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(V.VbdrError):
        sk.scan_slice(pairs[1:7])  # misaligned pointer
    with pytest.raises(V.VbdrError):
        sk.set_tuning(scan_defer=3)
    with pytest.raises(ValueError):
        sk.scan_slice(pairs.cpu())
    with pytest.raises(V.VbdrError):
        sk.load_state({"dr": np.zeros((5000, sk.L), np.uint8), "reg": np.zeros(5000, np.uint8),
                       "hist": np.zeros(33, np.uint64), "t": 0})  # histogram does not sum to m
    with pytest.raises(V.VbdrError):
        sk.load_state({"dr": np.zeros((5000, sk.L), np.uint8), "reg": np.zeros(5000, np.uint8),
                       "hist": np.array([4999, 1] + [0] * 31, np.uint64), "t": 0})  # not the registers' histogram
