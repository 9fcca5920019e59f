"""Brute-force pins for the oracle, written independently of it in numpy.

Nothing here follows the oracle's incremental update rules.  Registers are
recomputed from scratch as a fresh HyperLogLog over the pairs of the last k
closed slices, and distance recorders from closed forms over the whole slice
history.  The per-pair hash is a separate numpy implementation of
MurmurHash3_x86_32 that the published test vectors pin
(tests/golden/murmur3_x86_32.txt).

Conventions shared with the oracle (readings of arXiv:1810.13132):
  b = log2 g, L = 33 - b LBP1 values, one-byte DRs saturating at 255,
  H(x, N, A) = (murmur3(x, A) * N) >> 32, A0/A1 = low/high half of
  SplitMix64(hash_seed), bip hashed with A1, virtual seeds with A0.
"""
import numpy as np

SAT = 255
M32 = 0xFFFFFFFF


def murmur3_u32(x, seed):
    """MurmurHash3_x86_32 of the 4-byte little-endian keys x (uint32 array)."""
    x = np.asarray(x, dtype=np.uint32)
    seed = np.asarray(seed, dtype=np.uint32)
    with np.errstate(over="ignore"):
        k = x * np.uint32(0xCC9E2D51)
        k = (k << np.uint32(15)) | (k >> np.uint32(17))
        k = k * np.uint32(0x1B873593)
        h = seed ^ k
        h = (h << np.uint32(13)) | (h >> np.uint32(19))
        h = h * np.uint32(5) + np.uint32(0xE6546B64)
        h = h ^ np.uint32(4)
        h = h ^ (h >> np.uint32(16))
        h = h * np.uint32(0x85EBCA6B)
        h = h ^ (h >> np.uint32(13))
        h = h * np.uint32(0xC2B2AE35)
        h = h ^ (h >> np.uint32(16))
    return h.astype(np.uint32)


def splitmix64(state: int):
    state = (state + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & ((1 << 64) - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & ((1 << 64) - 1)
    return z ^ (z >> 31), state


def seeds(hash_seed: int):
    x, _ = splitmix64(hash_seed)
    return x & M32, x >> 32


def reduce_range(h, N: int):
    return ((np.asarray(h, dtype=np.uint64) * np.uint64(N)) >> np.uint64(32)).astype(np.uint64)


def rho_of(w, b: int):
    """Leftmost-1 position (from 1) within the top 32-b bits of w; 33-b if none."""
    w = np.asarray(w, dtype=np.uint64)
    out = np.full(w.shape, 33 - b, dtype=np.int64)
    for pos in range(32 - b, 0, -1):  # smallest position wins: assign last
        bit = (w >> np.uint64(32 - pos)) & np.uint64(1)
        out = np.where(bit == 1, pos, out)
    return out


def pair_map(pairs, m: int, g: int, hash_seed: int):
    """(pidx, rho) of every pair, straight from the definitions."""
    pairs = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    b = int(g).bit_length() - 1
    A0, A1 = seeds(hash_seed)
    bh = murmur3_u32(pairs[:, 1], A1).astype(np.uint64)
    vidx = (bh >> np.uint64(32 - b)).astype(np.uint32)
    w = (bh << np.uint64(b)) & np.uint64(M32)
    s1 = murmur3_u32(vidx, A0)
    pidx = reduce_range(murmur3_u32(pairs[:, 0], s1), m).astype(np.int64)
    return pidx, rho_of(w, b)


def host_pidx(aip: int, m: int, g: int, hash_seed: int):
    A0, _ = seeds(hash_seed)
    s1 = murmur3_u32(np.arange(g, dtype=np.uint32), A0)
    return reduce_range(murmur3_u32(np.full(g, aip, dtype=np.uint32), s1), m).astype(np.int64)


def fresh_registers(slices, m, g, k, hash_seed):
    """HyperLogLog registers of the pool built only from the last k closed slices."""
    reg = np.zeros(m, dtype=np.int64)
    for pairs in slices[max(0, len(slices) - k):]:
        p, r = pair_map(pairs, m, g, hash_seed)
        np.maximum.at(reg, p, r)
    return reg.astype(np.uint8)


def fresh_pcsa_runs(slices, m, g, k, hash_seed):
    """PCSA reading of the pool over the last k closed slices: the bitmap of
    BDR p holds every LBP1 seen there; the run is the number of consecutive
    set bits from LBP1 1."""
    b = int(g).bit_length() - 1
    L = 33 - b
    seen = np.zeros((m, L + 2), dtype=bool)
    for pairs in slices[max(0, len(slices) - k):]:
        p, r = pair_map(pairs, m, g, hash_seed)
        seen[p, r] = True
    run = np.zeros(m, dtype=np.int64)
    alive = np.ones(m, dtype=bool)
    for r in range(1, L + 1):
        alive &= seen[:, r]
        run += alive
    return run.astype(np.uint8)


def closed_form_dr(slices, m, g, hash_seed, layout: str):
    """Distance recorders after closing every slice in ``slices``.

    small layout: every LBP1 seen in slice s leaves DR = (T+1) - s;
    fast / serial: only the slice's maximum LBP1 at a BDR is recorded, and
    leaves DR = T - s; saturated at 255; never recorded -> 255.
    Returned canonically as dr[p, i-1]."""
    b = int(g).bit_length() - 1
    L = 33 - b
    T = len(slices) - 1
    last = np.full((m, L + 1), -1, dtype=np.int64)
    for s, pairs in enumerate(slices):
        p, r = pair_map(pairs, m, g, hash_seed)
        if layout == "small":
            last[p, r] = s
        else:
            mx = np.zeros(m, dtype=np.int64)
            np.maximum.at(mx, p, r)
            nz = np.nonzero(mx)[0]
            last[nz, mx[nz]] = s
    off = T + 1 if layout == "small" else T
    dist = np.where(last >= 0, off - last, SAT)
    return np.minimum(dist, SAT)[:, 1:].astype(np.uint8)


def open_slice_bits(pairs, m, g, hash_seed):
    """Fast layout bsLBP1 and serial nowLBP1 of an open slice."""
    p, r = pair_map(pairs, m, g, hash_seed)
    bs = np.zeros(m, dtype=np.uint64)
    np.bitwise_or.at(bs, p, (np.uint64(1) << (r - 1).astype(np.uint64)))
    now = np.zeros(m, dtype=np.int64)
    np.maximum.at(now, p, r)
    return bs.astype(np.uint32), now.astype(np.uint8)


def exact_cardinality(slices, aip):
    """|OP(aip)| over the given slices (Definition 1), by sets."""
    seen = set()
    for pairs in slices:
        pairs = np.asarray(pairs).reshape(-1, 2)
        seen.update(pairs[pairs[:, 0] == aip, 1].tolist())
    return len(seen)
