"""Window state of a VBDR pool in closed form -- TEST INFRASTRUCTURE.

Only tests may import this module.  It is a second formulation of the same
state as the step-by-step oracle (vbdr_oracle.c), for pools too large for
that one to slide every recorder of every slice in test time (2^26 BDRs
over a window of 60 slices and more).

Sec. 3 defines a distance recorder (DR) by what it holds: the number of
slices since its LBP1 value was last recorded in its BDR.  Recording sets it
to 0 (SetDR), every slice adds one (SlideDR), up to the saturation value.
The whole pool after t closed slices therefore follows from one number per
(BDR, LBP1): the slice of its last record.  This module keeps that number
and derives from it:
  * DR = min(sat, age), with the age counted as each layout counts it.
    Small layout (Alg. 9 records every pair's LBP1; Alg. 8 slides at the
    close, after the window is read): a record in slice s has age t - s
    after t closed slices.  Fast layout (Alg. 7 keeps a bit per LBP1, Alg. 6
    folds only the slice's highest one and sets that DR after the slide):
    only the slice maximum is recorded, with age t - 1 - s.  Packed layout:
    the small layout with LBP1 values above Lc recorded at Lc and
    saturation at 2^z - 1, z = ceil(log2(k+1)); recorders above Lc read
    saturated.  Never recorded: the initial value, sat.
  * The register of a BDR over the window of the k most recently closed
    slices (Alg. 2: the largest LBP1 whose DR is active): the largest LBP1
    recorded there in slices t-k .. t-1, 0 if none (capped at Lc).
  * The pool histogram of the registers.
The pair -> (pidx, LBP1) map is the oracle's own (getPhyIdx of Alg. 3 and
the bip hash of Alg. 4, vbdro_map_pairs).  Records of the open slice are
held until the advance closes it.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import oracle

_THREADS = 8


def map_pairs(m: int, g: int, hash_seed: int, pairs: np.ndarray):
    """oracle.map_pairs over chunks of the pairs in threads (the C mapping
    releases the interpreter lock); identical result."""
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    if n < (1 << 20):
        return oracle.map_pairs(m, g, hash_seed, pairs)
    cuts = np.linspace(0, n, _THREADS + 1).astype(np.int64)
    with ThreadPoolExecutor(_THREADS) as ex:
        parts = list(ex.map(lambda ab: oracle.map_pairs(m, g, hash_seed, pairs[ab[0]:ab[1]]),
                            zip(cuts[:-1], cuts[1:])))
    return np.concatenate([p for p, _ in parts]), np.concatenate([r for _, r in parts])


class WindowReplay:
    """One pool followed slice by slice through the slice of each
    (BDR, LBP1)'s last record.  layout: "fast", "small" or "packed"."""

    def __init__(self, m: int, g: int, k: int, hash_seed: int, layout: str, Lc: int = 0):
        if layout not in ("fast", "small", "packed"):
            raise ValueError(layout)
        b = int(g).bit_length() - 1
        if g != 1 << b or not 2 <= g <= 65536 or not g < m < 2**32 or not 1 <= k <= 254:
            raise ValueError("bad parameters")
        self.m, self.g, self.k, self.seed, self.layout = m, g, k, hash_seed, layout
        self.L = 33 - b
        self.Lc = self.L
        self.sat = 255
        if layout == "packed":
            if not 1 <= Lc <= self.L:
                raise ValueError("Lc out of range")
            z = 1
            while (1 << z) - 1 < k:
                z += 1
            self.Lc, self.sat = Lc, (1 << z) - 1
        # last[p, r-1] = 1 + the slice of the last record of LBP1 r at BDR p, 0 = never
        self.last = np.zeros((m, self.L), dtype=np.uint16)
        self.t = 0
        self._open = []

    def scan(self, pairs: np.ndarray):
        self.scan_mapped(*map_pairs(self.m, self.g, self.seed, pairs))

    def scan_mapped(self, pidx: np.ndarray, rho: np.ndarray):
        """Scan pairs already mapped to (pidx, LBP1) by map_pairs with this
        replay's m, g and hash seed."""
        if len(pidx):
            self._open.append((pidx, rho))

    def advance(self):
        """Close the open slice (slice number t)."""
        if self.t + 1 >= 1 << 16:
            raise ValueError("too many slices")
        stamp = np.uint16(self.t + 1)
        flat = self.last.reshape(-1)
        W = self.L
        if self._open:
            pidx = np.concatenate([p for p, _ in self._open]).astype(np.int64)
            rho = np.concatenate([r for _, r in self._open]).astype(np.int64)
            if self.layout == "fast":
                top = np.zeros(self.m, dtype=np.uint8)
                np.maximum.at(top, pidx, rho.astype(np.uint8))
                hit = np.flatnonzero(top)
                flat[hit * W + top[hit].astype(np.int64) - 1] = stamp
            else:
                flat[pidx * W + np.minimum(rho, self.Lc) - 1] = stamp
        self._open = []
        self.t += 1

    def registers(self, Lc: int = 0) -> np.ndarray:
        """(m,) uint8: largest LBP1 recorded in the last k closed slices
        (capped at Lc when given)."""
        return self.state(Lc=Lc, with_dr=False)["reg"]

    def state(self, Lc: int = 0, with_dr: bool = True) -> dict:
        """Canonical closed state after the last advance, in the form the
        oracle's and the library's exports take: dr (m, L) uint8, reg (m,),
        hist (33,) uint64, t.

        Lc > 0 on a small-layout replay gives the packed layout's state with
        Lc recorders instead (same records, LBP1 values above Lc merged into
        recorder Lc, z-bit saturation) without a replay of its own."""
        if self._open:
            raise ValueError("state() reads closed slices only: advance first")
        sat, cap = self.sat, self.Lc
        if Lc:
            if self.layout != "small" or not 1 <= Lc <= self.L:
                raise ValueError("a packed view needs a small-layout replay and 1 <= Lc <= L")
            z = 1
            while (1 << z) - 1 < self.k:
                z += 1
            sat, cap = (1 << z) - 1, Lc
        base = self.t if self.layout == "fast" else self.t + 1  # DR = base - stamp
        lo = max(self.t - self.k, 0) + 1  # stamps of the window's slices t-k .. t-1
        dr = np.empty((self.m, self.L), dtype=np.uint8) if with_dr else None
        reg = np.empty(self.m, dtype=np.uint8)
        oracle.lib().vbdro_replay_state(self.last.ctypes.data, self.m, self.L, cap, sat, base, lo,
                                        None if dr is None else dr.ctypes.data, reg.ctypes.data)
        hist = np.bincount(reg, minlength=oracle.NBINS).astype(np.uint64)
        return {"dr": dr, "reg": reg, "hist": hist, "t": self.t}
