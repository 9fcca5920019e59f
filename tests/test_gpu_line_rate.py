"""The line-rate workload's shape on the device, against the oracle.

Pool m = 2^26 BDRs, g = 1024 (b = 10, L = 23), window k = 60: the sketch
shape the benchmark times, in the configuration it times (deferred scans,
the deferred advance for the byte layouts, the packed advance at Lc = 16
and z = 6, the LDS-tiled estimate with 2^18-register tiles and blocks of
2^19 hosts).  The stream is the line-rate workload's (2^20 hosts,
Zipf(1.2) opposite sets on 1..10^6, Poisson(3) repeats, 20 % churn per
slice) at 2^22 pairs per slice, over k + 2 = 62 slices, so that slices 0
and 1 leave the window (Sec. 2.3, W(t, k)) and the DRs they set move past
the activity threshold.  Slice k carries 2^27 pairs, two full line-rate
slices scanned in two calls: records arrive at 2^16 per run of 2^15 BDRs on
average, the run capacity, so about half of the runs overflow and their
remaining records are applied by the scan itself (Alg. 7 / Alg. 9 directly);
the advance after it cannot trust its saturation masks.

Expected values come from the oracle: its pair map, its closed-form window
state (oracle/replay.py, pinned against the step-by-step oracle) and its
estimate of Alg. 5 over the closed-form registers.  BDR state (every DR,
register and histogram bin) must match bit for bit; estimates within 1e-6
relative plus the cancellation floor of the noise removal.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_13132_amd import vbdr
    vbdr.lib()
    return vbdr


def _assert_state(gs, exp, name, t):
    assert gs["t"] == exp["t"] == t + 1, name
    bad = np.argwhere(gs["dr"] != exp["dr"])
    assert len(bad) == 0, f"{name}: {len(bad)} DRs differ after slice {t}, first {bad[:4].tolist()}"
    assert not gs["bs"].any(), name
    assert np.array_equal(gs["reg"], exp["reg"]), f"{name}: registers differ after slice {t}"
    assert np.array_equal(gs["hist"], exp["hist"]), f"{name}: pool histogram differs after slice {t}"


def _assert_estimates(O, out, ref, raw, hist, m, g, what):
    em = O.hll_from_hist(hist, m)
    floor = 1e-12 * (m * np.abs(raw) + g * em) / (m - g)
    err = np.abs(out.astype(np.float64) - ref.astype(np.float64))
    bad = err > 1e-6 * np.abs(ref.astype(np.float64)) + floor
    assert not bad.any(), f"{what}: {int(bad.sum())} estimates off, e.g. {out[bad][:4]} vs {ref[bad][:4]}"


@pytest.mark.timeout(900)
def test_line_rate_shape_against_oracle(V):
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from oracle import replay
    from paper_1810_13132_amd import synth

    w = synth.LINE_RATE.scaled(pairs_per_slice=1 << 22)
    full = synth.LINE_RATE
    m, g, k, seed, Lc = w.m, w.g, w.k, w.seed, 16
    st, st_full = synth.Stream(w), synth.Stream(full)
    assert np.array_equal(st.aip, st_full.aip)
    torch.cuda.set_device(0)
    sks = {"fast": V.Sketch(m, g, k, seed, "fast"), "small": V.Sketch(m, g, k, seed, "small"),
           "packed": V.Sketch(m, g, k, seed, "packed", Lc=Lc)}
    for name, sk in sks.items():
        info = sk.info()
        assert info.scan_deferred == 1 and info.est_tiled == 1, name
        assert sk.L == 23 and sk.dr_bits == (6 if name == "packed" else 8)
    rp = {"fast": replay.WindowReplay(m, g, k, seed, "fast"), "small": replay.WindowReplay(m, g, k, seed, "small")}

    def expected(name):
        return rp["small"].state(Lc=Lc) if name == "packed" else rp[name].state()

    t0 = time.time()
    active = []
    n_slices = k + 2
    for t in range(n_slices):
        counts = np.zeros(w.hosts, dtype=np.uint32)
        if t == k:
            c2 = np.zeros(w.hosts, dtype=np.uint32)
            parts = [st_full.slice(t, host_pairs=counts), st_full.slice(t + 1000, host_pairs=c2)]
            counts += c2
        else:
            parts = [st.slice(t, host_pairs=counts)]
        active.append(counts > 0)
        active = active[-k:]
        for pairs in parts:
            pd = V.to_device_u32(pairs.reshape(-1))
            for sk in sks.values():
                sk.scan_slice(pd)
            pidx, rho = replay.map_pairs(m, g, seed, pairs)
            for r in rp.values():
                r.scan_mapped(pidx, rho)
            torch.cuda.synchronize()
            del pd
        for sk in sks.values():
            sk.advance_slice()
        for r in rp.values():
            r.advance()
        if t in (k - 1, k + 1):
            for name, sk in sks.items():
                _assert_state(sk.state(), expected(name), name, t)
            _log(f"slice {t}: full state of 3 layouts equal ({time.time() - t0:.0f}s)")
        elif t in (0, k):
            reg_b = rp["small"].registers()
            assert np.array_equal(reg_b, rp["fast"].registers())
            reg_p = rp["small"].registers(Lc=Lc)
            for name, sk in sks.items():
                reg, hist = sk.registers()
                exp = reg_p if name == "packed" else reg_b
                assert np.array_equal(reg, exp), f"{name}: registers differ after slice {t}"
                assert np.array_equal(hist, np.bincount(exp, minlength=33).astype(np.uint64)), name
            _log(f"slice {t}: registers equal ({time.time() - t0:.0f}s)")

    # estimates over the window after slice k + 1: every host of the stream but
    # the last 3001, so the second block of 2^19 hosts ends in a partial sub-block
    n_est = w.hosts - 3001
    hosts = st.aip[:n_est]
    hd = V.to_device_u32(hosts)
    outs = {}
    for name, sk in sks.items():
        tiled = sk.estimate(hd).cpu().numpy()
        sk.set_tuning(est_binned=2)
        assert sk.info().est_tiled == 0
        parted = sk.estimate(hd).cpu().numpy()
        sk.set_tuning()
        assert sk.info().est_tiled == 1
        assert np.array_equal(tiled, parted), f"{name}: tiled and partitioned estimates differ"
        outs[name] = tiled
    assert np.array_equal(outs["fast"], outs["small"])

    act = np.flatnonzero(np.logical_or.reduce(active)[:n_est])
    assert len(act) >= 1 << 17
    rng = np.random.default_rng(62)
    edges = np.concatenate([np.arange(64), np.arange((1 << 19) - 64, (1 << 19) + 64), np.arange(n_est - 64, n_est)])
    sample = np.unique(np.concatenate([rng.choice(act, 1 << 17, replace=False), edges]))
    reg_b, reg_p = rp["small"].registers(), rp["small"].registers(Lc=Lc)
    with ThreadPoolExecutor(2) as ex:
        fb = ex.submit(O.estimate_registers, m, g, seed, reg_b, hosts[sample], True, True)
        fp = ex.submit(O.estimate_registers, m, g, seed, reg_p, hosts[sample], True)
        ref_b, raw_b, hist_b = fb.result()
        ref_p, raw_p = fp.result()
    pool_b = np.bincount(reg_b, minlength=33).astype(np.uint64)
    pool_p = np.bincount(reg_p, minlength=33).astype(np.uint64)
    for name in ("fast", "small"):
        _assert_estimates(O, outs[name][sample], ref_b, raw_b, pool_b, m, g, name)
    _assert_estimates(O, outs["packed"][sample], ref_p, raw_p, pool_p, m, g, "packed")
    # per-host histograms and raw E_s through the direct path
    ex_out, ex_raw, ex_hist = sks["small"].estimate_ex(V.to_device_u32(hosts[sample]))
    assert np.array_equal(ex_hist.cpu().numpy().astype(np.uint32), hist_b)
    np.testing.assert_allclose(ex_raw.cpu().numpy(), raw_b, rtol=1e-13, atol=0)
    assert np.array_equal(ex_out.cpu().numpy(), outs["small"][sample])
    _log(f"estimates of {n_est} hosts equal across paths; {len(sample)} ({len(act)} active) checked against "
         f"the oracle ({time.time() - t0:.0f}s)")
    for sk in sks.values():
        sk.close()
