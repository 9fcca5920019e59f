"""Replicas of one fast-layout sketch that scan disjoint shares of each slice
and exchange their per-slice max-LBP1 maps (export, element-wise MAX, import)
end every slice in the state of one sketch that scanned all the pairs (the
oracle's), bit for bit.  The exported map is checked against its definition:
the highest LBP1 of the slice's pairs at each BDR (the serial layout's
nowLBP1, Alg. 1 / Alg. 4), computed from the oracle's (pidx, LBP1) map of
each pair.  The MAX stands in for the all-reduce of a multi-GPU run."""
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


def _now_ref(O, m, g, seed, pairs):
    pidx, rho = O.map_pairs(m, g, seed, pairs)
    now = np.zeros(m, np.uint8)
    np.maximum.at(now, pidx.astype(np.int64), rho)
    return now


@pytest.mark.parametrize("m", [70001, (1 << 22) + 77])  # direct scans; deferred scans (large pool)
def test_replicas_merge_to_one_sketch(V, O, m):
    g, k, seed, P = 256, 3, 41, 3
    rng = np.random.default_rng(m % 1000)
    aips = rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)
    reps = [V.Sketch(m, g, k, seed, "fast") for _ in range(P)]
    assert reps[0].info().scan_deferred == (m >= 1 << 22)
    osk = O.Sketch(m, g, k, seed, O.GFAST)
    hosts = aips[:300]
    for t in range(5):
        n = 0 if t == 2 else int(rng.integers(1 << 16, 1 << 18))
        pairs = np.stack([aips[rng.integers(0, len(aips), n)],
                          rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)], 1).astype(np.uint32)
        share = rng.integers(0, P, n)
        nows = []
        for r, sk in enumerate(reps):
            mine = pairs[share == r]
            if len(mine):
                sk.scan_slice(V.to_device_u32(mine.reshape(-1)))
            now = sk.export_now()
            assert np.array_equal(now.cpu().numpy(), _now_ref(O, m, g, seed, mine)), f"replica {r} slice {t}"
            nows.append(now)
        merged = V.now_max(V.now_max(nows[0], nows[1]), nows[2])
        for sk in reps:
            sk.import_now(merged)
            sk.advance_slice()
        osk.scan(pairs)
        osk.advance()
        ref = osk.state()
        for r, sk in enumerate(reps):
            st = sk.state()
            for key in ("dr", "reg", "hist"):
                assert np.array_equal(st[key], ref[key]), (key, r, t)
    hd = V.to_device_u32(hosts)
    e0 = reps[0].estimate(hd)
    assert all(torch.equal(sk.estimate(hd), e0) for sk in reps[1:])


def test_small_layout_rejects_maps(V):
    sk = V.Sketch(5000, 16, 3, 1, "small")
    with pytest.raises(V.VbdrError):
        sk.export_now()
