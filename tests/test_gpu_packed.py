"""The packed layout (z-bit bit-sliced DRs, Lc recorders, Table 1's sizes)
against the oracle's packed layout, bit for bit: DRs after every scan (the
export applies pending records) and every advance, registers, histograms,
per-host register histograms; raw E_s within 1e-13 and estimates within the
bar of the other layouts (1e-6 relative plus the cancellation floor).  Every
case runs k + 4 slices, so DRs set in the first slices leave the window and
reach the saturation value 2^z - 1 on the device.  Cases cover z = 1..8, Lc
below and at L, a pool of one tile with more records than a tile's run holds
(the direct update path), empty slices and a resume from an exported state."""
import numpy as np
import pytest

from test_gpu_parity import assert_estimates_close

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


def _equal(sk, osk, where):
    a, b = sk.state(), osk.state()
    for key in ("dr", "reg", "hist"):
        assert np.array_equal(a[key], b[key]), (key, where, np.argwhere(a[key] != b[key])[:3] if a[key].ndim else None)


@pytest.mark.parametrize("m,g,k,Lc_off,n_max", [
    (5003, 16, 1, 0, 40000),         # z = 1; one tile
    (5003, 16, 3, 20, 200000),       # z = 2, Lc = 9; more records than the tile's run: direct updates
    (70001, 64, 4, 0, 60000),        # z = 3, Lc = L; several tiles, ragged last
    (70001, 64, 60, 15, 60000),      # z = 6, Lc = 12
    (9000, 8, 254, 2, 20000),        # z = 8
    ((1 << 22) + 77, 256, 7, 9, 1 << 18),  # z = 3, Lc = 16, large pool
])
def test_packed_matches_oracle(V, O, m, g, k, Lc_off, n_max):
    rng = np.random.default_rng(m + k)
    L = 33 - (g.bit_length() - 1)
    Lc = L - Lc_off
    sk = V.Sketch(m, g, k, 7, "packed", Lc=Lc)
    osk = O.Sketch(m, g, k, 7, O.GPACKED, Lc=Lc)
    assert (sk.Lc, sk.dr_bits) == (Lc, int(np.ceil(np.log2(k + 1)))) and sk.info().scan_deferred == 1
    aips = rng.integers(0, 2**32, 500, dtype=np.uint64).astype(np.uint32)
    hosts = np.concatenate([aips[:200], np.array([0, 12345, 0xFFFFFFFF], np.uint32)])
    sat = (1 << sk.dr_bits) - 1
    dr0 = None
    for t in range(k + 4):
        n = 0 if t == 2 else int(rng.integers(n_max // 4, n_max))
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        if t == 1:  # a repeated pair: many identical records
            pairs[: n // 2] = pairs[0]
        pd = V.to_device_u32(pairs.reshape(-1))
        half = n // 2
        sk.scan_slice(pd[: 2 * half])
        osk.scan(pairs[:half])
        if t in (1, 3):
            _equal(sk, osk, f"mid-slice {t}")
        sk.scan_slice(pd[2 * half:])
        osk.scan(pairs[half:])
        sk.advance_slice()
        osk.advance()
        _equal(sk, osk, f"slice {t}")
        if t == 0:
            dr0 = osk.state()["dr"]
        if t in (k - 1, k, k + 3) or t % 16 == 5:
            assert_estimates_close(V, O, sk, osk, hosts)
    # DRs set in slice 0 have slid to saturation on the device (with z = 1 a
    # recorded DR reads 1 = 2^z - 1 from its first close on)
    dr_end = sk.state()["dr"]
    assert sat == 1 or ((dr0 < sat) & (dr_end == sat)).any()
    # resume
    b = V.Sketch(m, g, k, 7, "packed", Lc=Lc)
    b.load_state(sk.state())
    n = n_max // 2
    pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                      rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
    for s_ in (sk, b):
        s_.scan_slice(V.to_device_u32(pairs.reshape(-1)))
        s_.advance_slice()
    osk.scan(pairs)
    osk.advance()
    _equal(b, osk, "resumed")
    _equal(sk, osk, "continued")


def test_packed_memory_and_refusals(V):
    small = V.Sketch(1 << 22, 1024, 60, 1, "small")
    packed = V.Sketch(1 << 22, 1024, 60, 1, "packed", Lc=16)
    # DR state: 23 bytes per BDR against 16 recorders of 6 bits (12 bytes)
    assert small.info().state_bytes - packed.info().state_bytes >= (1 << 22) * (23 - 12)
    with pytest.raises(V.VbdrError):
        packed.set_tuning(scan_defer=2)
    with pytest.raises(V.VbdrError):
        packed.enable_pcsa(True)
    with pytest.raises(V.VbdrError):
        V.Sketch(1 << 22, 1024, 60, 1, "packed", Lc=24)
