"""LogLog and PCSA on the pool (the pool serves them too: the text after
Alg. 5, Sec. 5), HIP path vs oracle.  PCSA runs bit for bit after every
advance (direct and deferred scans); estimates within the HyperLogLog path's
bar: FP64 epilogues that differ only in the last bit of exp2/pow, so E_s to
1e-13 relative and the FP32 result to 1e-6 relative plus a floor for the
cancellation in (m E_s - g E_m)/(m - g)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _close(V, O, sk, osk, hosts, kind):
    hd = V.to_device_u32(hosts)
    out, raw = sk.estimate_kind(hd, kind, with_raw=True)
    out, raw = out.cpu().numpy(), raw.cpu().numpy()
    code = {"loglog": O.LOGLOG, "pcsa": O.PCSA}[kind]
    ref, ref_raw = osk.estimate_kind(hosts, code, with_raw=True)
    np.testing.assert_allclose(raw, ref_raw, rtol=1e-13, atol=0)
    m, g = float(osk.m), float(osk.g)
    floor = 1e-12 * (m * np.abs(ref_raw) + g * ref_raw.max()) / (m - g)
    bad = np.abs(out.astype(np.float64) - ref) > 1e-6 * np.abs(ref) + floor + 1e-6 * m * g / (m - g)
    assert not bad.any(), (kind, out[bad][:5], ref[bad][:5])


@pytest.mark.parametrize("m", [50021, (1 << 22) + 77])  # direct scans; deferred scans
def test_pcsa_and_loglog_match_oracle(V, O, m):
    g, k, seed = 128, 3, 51
    rng = np.random.default_rng(m % 997)
    aips = rng.integers(0, 2**32, 1500, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, "small")
    sk.enable_pcsa(True)
    with pytest.raises(V.VbdrError):  # no runs before an advance
        sk.estimate_kind(V.to_device_u32(aips[:4]), "pcsa")
    osk = O.Sketch(m, g, k, seed, O.GSMALL)
    hosts = np.concatenate([aips[:400], rng.integers(0, 2**32, 50, dtype=np.uint64).astype(np.uint32)])
    for t in range(5):
        n = 0 if t == 2 else int(rng.integers(1 << 16, 1 << 18))
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        if n:
            sk.scan_slice(V.to_device_u32(pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
        assert np.array_equal(sk.pcsa_registers(), osk.pcsa_registers()), t
        for kind in ("loglog", "pcsa"):
            _close(V, O, sk, osk, hosts, kind)
    # the HyperLogLog kind is the plain estimate
    hd = V.to_device_u32(hosts)
    assert torch.equal(sk.estimate_kind(hd, "hll"), sk.estimate(hd))


def test_loglog_on_fast_layout_and_pcsa_refused(V, O):
    m, g, k, seed = 30011, 64, 2, 3
    rng = np.random.default_rng(5)
    aips = rng.integers(0, 2**32, 300, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, "fast")
    osk = O.Sketch(m, g, k, seed, O.GFAST)
    pairs = np.stack([aips[rng.integers(0, 300, 50000)],
                      rng.integers(0, 2**32, 50000, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
    sk.scan_slice(V.to_device_u32(pairs.reshape(-1)))
    osk.scan(pairs)
    sk.advance_slice()
    osk.advance()
    _close(V, O, sk, osk, aips, "loglog")
    with pytest.raises(V.VbdrError):
        sk.enable_pcsa(True)
    with pytest.raises(V.VbdrError):
        sk.estimate_kind(V.to_device_u32(aips), "pcsa")


def test_failed_pcsa_allocation_leaves_sketch_whole(V):
    """An out-of-memory failure while enabling PCSA runs (either of its two
    allocations) returns VBDR_ENOMEM and leaves the sketch as it was: the
    LDS-tiled estimate's workspaces stay allocated and give the same
    estimates, PCSA stays off, and enabling it again afterwards works."""
    m, g, k = 1 << 24, 1024, 4
    rng = np.random.default_rng(77)
    aips = rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, 3, "small")
    assert sk.info().est_tiled == 1
    n = 1 << 20
    pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                      rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
    sk.scan_slice(V.to_device_u32(pairs.reshape(-1)))
    sk.advance_slice()
    hd = V.to_device_u32(aips)
    before = sk.estimate(hd)
    bytes0 = sk.info().state_bytes
    try:
        for after in (0, 1):  # the run array, then the pool sum
            V.fail_allocation_after(after)
            with pytest.raises(V.VbdrError) as e:
                sk.enable_pcsa(True)
            assert e.value.code == -2
            V.fail_allocation_after(-1)
            assert sk.info().state_bytes == bytes0 and sk.info().est_tiled == 1
            assert torch.equal(sk.estimate(hd), before)
            with pytest.raises(V.VbdrError) as e:
                sk.estimate_kind(hd, "pcsa")
            assert e.value.code == -4
    finally:
        V.fail_allocation_after(-1)
    sk.enable_pcsa(True)
    sk.advance_slice()
    assert sk.estimate_kind(hd, "pcsa").shape == (len(aips),)
    sk.close()
