"""Pins of the oracle's closed-form window state (oracle/replay.py) and of
its estimate over a given register array.

The replay derives DRs from the slice of each (BDR, LBP1)'s last record
(Sec. 3's definition of a DR) instead of sliding every DR every slice.  It
must agree, element by element, with the step-by-step oracle (Alg. 1/2/6/8/9
as written) and with the numpy brute force (its own hash implementation,
registers as a fresh HyperLogLog of the last k closed slices), for all
three GPU layouts, over histories long enough to saturate.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import bruteforce as B
from oracle import replay

CODES = {"fast": 1, "small": 2, "packed": 3}


def _slices(seed, n_slices, max_pairs, n_aip, n_bip, empty_prob=0.15):
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, n_aip, dtype=np.uint64).astype(np.uint32)
    bips = rng.integers(0, 2**32, n_bip, dtype=np.uint64).astype(np.uint32)
    out = []
    for _ in range(n_slices):
        n = 0 if rng.random() < empty_prob else int(rng.integers(1, max_pairs + 1))
        out.append(np.stack([aips[rng.integers(0, n_aip, n)], bips[rng.integers(0, n_bip, n)]], 1)
                   .astype(np.uint32).reshape(-1, 2))
    return aips, out


def _follow(O, layout, m, g, k, seed, slices, Lc=0, split=1):
    rp = replay.WindowReplay(m, g, k, seed, layout, Lc=Lc)
    osk = O.Sketch(m, g, k, seed, CODES[layout], Lc=Lc)
    view = replay.WindowReplay(m, g, k, seed, "small") if layout == "packed" else None
    for t, pairs in enumerate(slices):
        for part in np.array_split(pairs, split):
            rp.scan(part)
            if view:
                view.scan(part)
        osk.scan(pairs)
        rp.advance()
        osk.advance()
        if view:
            view.advance()
        b = osk.state()
        outs = [rp.state()] + ([view.state(Lc=Lc)] if view else [])
        for a in outs:
            assert a["t"] == b["t"] == t + 1
            assert np.array_equal(a["dr"], b["dr"]), (layout, t, np.argwhere(a["dr"] != b["dr"])[:4])
            assert np.array_equal(a["reg"], b["reg"]), (layout, t)
            assert np.array_equal(a["hist"], b["hist"]), (layout, t)
    return rp, osk


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31), b=st.integers(1, 7), k=st.integers(1, 10), m_extra=st.integers(1, 500),
       n_slices=st.integers(1, 14), max_pairs=st.integers(1, 300), n_aip=st.integers(1, 8),
       n_bip=st.integers(1, 80), layout=st.sampled_from(["fast", "small", "packed"]), lc_off=st.integers(0, 30))
def test_replay_equals_stepwise_oracle(oracle_mod, seed, b, k, m_extra, n_slices, max_pairs, n_aip, n_bip,
                                       layout, lc_off):
    g = 1 << b
    m = g + m_extra
    L = 33 - b
    Lc = max(1, L - lc_off) if layout == "packed" else 0
    _, slices = _slices(seed, n_slices, max_pairs, n_aip, n_bip)
    _follow(oracle_mod, layout, m, g, k, seed, slices, Lc=Lc, split=2)


@pytest.mark.parametrize("layout,k,Lc", [("fast", 5, 0), ("small", 5, 0), ("packed", 60, 20), ("packed", 254, 26),
                                         ("small", 254, 0)])
def test_replay_long_history(oracle_mod, layout, k, Lc):
    """300 slices: byte DRs reach 255, packed ones 2^z - 1, and stay."""
    m, g = 211, 64
    _, slices = _slices(9, 300, 40, 3, 200, empty_prob=0.6)
    rp, _ = _follow(oracle_mod, layout, m, g, k, 13, slices, Lc=Lc)
    dr = rp.state()["dr"]
    assert (dr == rp.sat).any() and (dr < rp.sat).any()


def test_replay_matches_bruteforce(oracle_mod):
    """The independent numpy closed forms (own hash, own pair map)."""
    m, g, k, seed = 3001, 32, 4, 21
    _, slices = _slices(4, 20, 500, 6, 400)
    for layout in ("fast", "small"):
        rp = replay.WindowReplay(m, g, k, seed, layout)
        for t, pairs in enumerate(slices):
            rp.scan(pairs)
            rp.advance()
            s = rp.state()
            assert np.array_equal(s["dr"], B.closed_form_dr(slices[: t + 1], m, g, seed, layout))
            assert np.array_equal(s["reg"], B.fresh_registers(slices[: t + 1], m, g, k, seed))


def test_replay_threaded_map_is_the_oracle_map(oracle_mod):
    rng = np.random.default_rng(5)
    pairs = rng.integers(0, 2**32, ((1 << 20) + 77, 2), dtype=np.uint64).astype(np.uint32)
    p1, r1 = replay.map_pairs(1 << 26, 1024, 3, pairs)
    sub = pairs[::4099]
    p2, r2 = oracle_mod.map_pairs(1 << 26, 1024, 3, sub)
    assert np.array_equal(p1[::4099], p2) and np.array_equal(r1[::4099], r2)
    assert len(p1) == len(pairs)


def test_replay_rejects_open_state(oracle_mod):
    rp = replay.WindowReplay(1000, 16, 3, 1, "small")
    rp.scan(np.array([[1, 2]], np.uint32))
    with pytest.raises(ValueError):
        rp.state()


def test_estimate_registers_is_the_sketch_estimate(oracle_mod):
    """Alg. 5 over a register array given by the caller equals the sketch's
    own estimate when given that sketch's registers."""
    O = oracle_mod
    m, g, k, seed = 5003, 64, 3, 8
    aips, slices = _slices(6, 6, 3000, 20, 2000)
    osk = O.Sketch(m, g, k, seed, O.GSMALL)
    for pairs in slices:
        osk.scan(pairs)
        osk.advance()
    hosts = np.concatenate([aips, np.array([0, 7, 0xFFFFFFFF], np.uint32)])
    ref, ref_raw, ref_hist = osk.estimate(hosts, with_raw=True, with_hist=True)
    out, raw, hist = O.estimate_registers(m, g, seed, osk.state()["reg"], hosts, with_raw=True, with_hist=True)
    assert np.array_equal(out, ref) and np.array_equal(raw, ref_raw) and np.array_equal(hist, ref_hist)
    bad = osk.state()["reg"].copy()
    bad[3] = 40
    with pytest.raises(ValueError):
        O.estimate_registers(m, g, seed, bad, hosts)
