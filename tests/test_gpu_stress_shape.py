"""The stress workload's sketch shape on the device, against the oracle.

Pool m = 2^24 BDRs, g = 2048 (b = 11, L = 22), window k = 128: the shape
the stress benchmark times.  Deferred scans and advances; the LDS-tiled
estimate with 2^16-register tiles, two seeds per thread in its first pass
(g is twice the pass's workgroup) and blocks of 2^18 hosts; the packed
layout at Lc = 16 recorders of z = 8 bits.  k = 128 is the
edge of the advance's bit-7 activity test: the fast layout's threshold
k - 1 = 127 takes it, the small layout's threshold k = 128 takes the
general comparison.  The stream is the stress workload's (Zipf(1.5)
opposite sets, 16 planted heavy hosts) at 2^20 pairs per slice over k + 2
slices, so that slices 0 and 1 leave the window (Sec. 2.3, W(t, k)).

Expected values come from the oracle's pair map and closed-form window
state (oracle/replay.py) and its estimate of Alg. 5 over those registers.
BDR state must match bit for bit; estimates within 1e-6 relative plus the
cancellation floor of the noise removal.
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


@pytest.mark.timeout(900)
def test_stress_shape_against_oracle(V):
    from oracle import oracle as O
    from oracle import replay
    from paper_1810_13132_amd import synth

    w = synth.STRESS.scaled(pairs_per_slice=1 << 20)
    m, g, k, seed = w.m, w.g, w.k, w.seed
    st = synth.Stream(w)
    torch.cuda.set_device(0)
    Lc = 16
    sks = {"fast": V.Sketch(m, g, k, seed, "fast"), "small": V.Sketch(m, g, k, seed, "small"),
           "packed": V.Sketch(m, g, k, seed, "packed", Lc=Lc)}
    for name, sk in sks.items():
        info = sk.info()
        assert info.scan_deferred == 1 and info.est_tiled == 1, name
        assert sk.L == 22 and sk.dr_bits == 8, name  # k = 128 needs z = 8 bits in the packed layout too
    rp = {name: replay.WindowReplay(m, g, k, seed, name) for name in ("fast", "small")}

    def expected(name):
        return rp["small"].state(Lc=Lc) if name == "packed" else rp[name].state()

    t0 = time.time()
    last_seen = np.full(w.hosts, -1, dtype=np.int32)  # last slice with a pair of the host
    n_slices = k + 2
    for t in range(n_slices):
        counts = np.zeros(w.hosts, dtype=np.uint32)
        pairs = st.slice(t, host_pairs=counts)
        last_seen[counts > 0] = t
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
                gs, exp = sk.state(), expected(name)
                assert gs["t"] == exp["t"] == t + 1, name
                bad = np.argwhere(gs["dr"] != exp["dr"])
                assert len(bad) == 0, f"{name}: {len(bad)} DRs differ after slice {t}, first {bad[:4].tolist()}"
                assert not gs["bs"].any(), name
                assert np.array_equal(gs["reg"], exp["reg"]), f"{name}: registers differ after slice {t}"
                assert np.array_equal(gs["hist"], exp["hist"]), f"{name}: pool histogram differs after slice {t}"
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

    # the hosts with a pair in the window (slices 2 .. k + 1), in stream order
    act = np.flatnonzero(last_seen >= n_slices - k)
    assert len(act) > 1 << 18, len(act)  # more than one block of the tiled estimate
    hosts = st.aip[act]
    hd = V.to_device_u32(hosts)
    outs = {}
    for name, sk in sks.items():
        tiled = sk.estimate(hd).cpu().numpy()
        sk.set_tuning(est_binned=2)
        assert sk.info().est_tiled == 0
        parted = sk.estimate(hd).cpu().numpy()
        sk.set_tuning()
        assert np.array_equal(tiled, parted), f"{name}: tiled and partitioned estimates differ"
        outs[name] = tiled
    assert np.array_equal(outs["fast"], outs["small"])

    rng = np.random.default_rng(130)
    n = len(act)
    # the tiled estimate splits the hosts into blocks of equal size (whole sub-blocks of 2048), at most 2^18
    nblk = -(-n // (1 << 18))
    blk = -(-(-(-n // nblk)) // 2048) * 2048
    edges = np.concatenate([np.arange(64), np.arange(blk - 64, blk + 64), np.arange(n - 64, n)])
    heavy = np.flatnonzero(np.isin(hosts, st.aip[np.argsort(st.n)[-16:]]))  # the planted heavy hosts
    sample = np.unique(np.concatenate([rng.choice(n, 1 << 14, replace=False), edges, heavy]))
    reg = rp["small"].registers()
    ref, raw, hist = O.estimate_registers(m, g, seed, reg, hosts[sample], True, True)
    reg_p = rp["small"].registers(Lc=Lc)
    ref_p, raw_p = O.estimate_registers(m, g, seed, reg_p, hosts[sample], True)

    def check(name, ref, raw, reg):
        em = O.hll_from_hist(np.bincount(reg, minlength=33).astype(np.uint64), m)
        floor = 1e-12 * (m * np.abs(raw) + g * em) / (m - g)
        got = outs[name][sample].astype(np.float64)
        bad = np.abs(got - ref.astype(np.float64)) > 1e-6 * np.abs(ref.astype(np.float64)) + floor
        assert not bad.any(), f"{name}: {int(bad.sum())} estimates off, e.g. {got[bad][:4]} vs {ref[bad][:4]}"

    check("fast", ref, raw, reg)
    check("small", ref, raw, reg)
    check("packed", ref_p, raw_p, reg_p)
    ex_out, ex_raw, ex_hist = sks["small"].estimate_ex(V.to_device_u32(hosts[sample]))
    assert np.array_equal(ex_hist.cpu().numpy().astype(np.uint32), hist)
    np.testing.assert_allclose(ex_raw.cpu().numpy(), raw, rtol=1e-13, atol=0)
    _log(f"estimates of {n} active hosts equal across paths; {len(sample)} checked against the oracle "
         f"({time.time() - t0:.0f}s)")
    for sk in sks.values():
        sk.close()
