"""vbdr_estimate_noalloc, the estimate for callers that cannot allocate,
against vbdr_estimate through the C ABI: bit-identical outputs on two calls
in a row, the second with fewer hosts, for a pool that takes the
partitioned estimate (its partial sums then live in the library's static
scratch, 65536 hosts per pass, so 70001 hosts take two passes) and for a
small pool that takes the direct estimate.  The static array keeps the
previous call's sums; the second, smaller call must not read them."""
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


def _fill(V, sk, seed, n_slices, n_pairs, n_aip):
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, n_aip, dtype=np.uint64).astype(np.uint32)
    for _ in range(n_slices):
        pairs = np.stack([aips[rng.integers(0, n_aip, n_pairs)],
                          rng.integers(0, 2**32, n_pairs, dtype=np.uint64).astype(np.uint32)], 1)
        sk.scan_slice(V.to_device_u32(pairs.astype(np.uint32).reshape(-1)))
        sk.advance_slice()
    return aips


@pytest.mark.parametrize("m,g,k,layout,n1,n2", [
    ((1 << 22) + 77, 256, 3, "small", 70001, 1000),   # partitioned: two passes, then one
    ((1 << 24), 1024, 5, "fast", 66000, 65536),        # tiled by default; the static path partitions
    (50000, 64, 4, "small", 3000, 17),                 # direct estimate, no scratch
])
def test_noalloc_estimate_equals_estimate(V, m, g, k, layout, n1, n2):
    sk = V.Sketch(m, g, k, 11, layout)
    aips = _fill(V, sk, m % 1000, 3, 1 << 18, 4000)
    rng = np.random.default_rng(5)
    for n in (n1, n2):
        hosts = np.concatenate([aips, rng.integers(0, 2**32, max(n - len(aips), 0), dtype=np.uint64)
                                .astype(np.uint32)])[:n]
        hd = V.to_device_u32(hosts)
        ref = sk.estimate(hd).cpu().numpy()
        out = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        sk.estimate_noalloc(hd, out)
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), f"n={n}: {np.flatnonzero(got != ref)[:5]}"
        assert (ref[: min(n, 4000)] > 0).any()
    sk.close()


def test_noalloc_estimate_argument_errors(V):
    sk = V.Sketch((1 << 22) + 77, 256, 3, 1, "small")
    hd = V.to_device_u32(np.arange(10, dtype=np.uint32))
    with pytest.raises(ValueError):
        sk.estimate_noalloc(hd, torch.empty(9, dtype=torch.float32, device="cuda"))
    lib = V.lib()
    assert lib.vbdr_estimate_noalloc(None, hd.data_ptr(), 10, hd.data_ptr(), None) == -1
    assert lib.vbdr_estimate_noalloc(sk._h, None, 10, None, None) == -1
    assert lib.vbdr_estimate_noalloc(sk._h, hd.data_ptr(), 1 << 40, hd.data_ptr(), None) == -1
    assert lib.vbdr_estimate_noalloc(sk._h, None, 0, None, None) == 0
    sk.close()
