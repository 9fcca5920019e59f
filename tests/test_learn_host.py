"""Host-side pieces of the learned-estimator driver (no GPU): the exact window
truth used as training target, checked against Definition 1 by sets."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_window_truth_matches_sets():
    from paper_1810_13132_amd import learn
    import bruteforce as B
    rng = np.random.default_rng(0)
    aips = rng.integers(0, 2**32, 40, dtype=np.uint64).astype(np.uint32)
    aips[:5] = [0, 1, 2**31, 2**32 - 1, 2**31 - 1]  # both halves of the address space
    slices = []
    for _ in range(3):
        n = 5000
        pairs = np.stack([aips[rng.integers(0, 40, n)],
                          rng.integers(0, 300, n).astype(np.uint32) * np.uint32(2654435761)], 1).astype(np.uint32)
        slices.append(pairs)
    keys = []
    for p in slices:
        t = torch.from_numpy(p.view(np.int32)).to(torch.int64) & 0xFFFFFFFF
        keys.append((t[:, 0] << 32) | t[:, 1])
    hosts = np.concatenate([aips, np.array([12345], np.uint32)])
    got = learn.window_truth(keys, torch.from_numpy(hosts.astype(np.int64))).numpy()
    ref = [B.exact_cardinality(slices, int(h)) for h in hosts]
    assert got.tolist() == ref


def test_stress_window_generators():
    """The synthetic stress windows plant hosts whose truth is their count of
    opposite hosts: the keyed map must be a bijection of 32-bit values (so a
    host's opposite hosts are distinct), and the int32 view must keep the 32
    bits of every value."""
    from paper_1810_13132_amd import learn
    x = torch.arange(0, 1 << 20, dtype=torch.int64)
    for key in (0, 12345, 2**32 - 1):
        y = learn._bijection32(x, key)
        assert int(y.min()) >= 0 and int(y.max()) < 2**32
        assert len(torch.unique(y)) == len(x)
    # a full 16-bit slice of the input space maps one to one as well
    hi = torch.arange(0, 1 << 16, dtype=torch.int64) << 16
    assert len(torch.unique(learn._bijection32(hi, 7))) == 1 << 16
    v = torch.tensor([0, 1, 2**31 - 1, 2**31, 2**32 - 1], dtype=torch.int64)
    got = learn._as_i32(v)
    assert got.dtype == torch.int32
    assert (got.to(torch.int64) & 0xFFFFFFFF).tolist() == v.tolist()
