"""Seeded synthetic (aip, bip) pair streams shaped like edge-router traffic.

Input generation only (no hashing, mapping or counting of the estimator);
both the HIP path and the CPU oracle consume what this module emits.  The
stream model is described in synth.c.  Workload presets:

* ``TINY``      -- 2^12 hosts, Zipf(1.1) opposite sets on 1..10^4, 2^20 pairs
                   per slice, 12 slices; sketch m=2^18, g=256, k=4.
* ``LINE_RATE`` -- 2^20 hosts, Zipf(1.2) on 1..10^6, 2^26 pairs per slice,
                   64 slices; sketch m=2^26, g=1024, k=60.
* ``MID``       -- 2^14 hosts, Zipf(1.1) on 1..10^4, 2^22 pairs per slice,
                   24 slices; sketch m=2^20, g=512, k=16 (the size of a
                   typical member of the batched workload).
* ``STRESS``    -- 2^24 hosts, 16 planted heavy hosts with 10^6..10^7
                   opposite hosts, Zipf(1.5) on 1..10^4 elsewhere, 2^27
                   pairs per slice; sketch m=2^24, g=2048, k=128.

Every stream repeats each (aip, bip) unit Poisson(3) times and replaces 20%
of every host's opposite set per slice.
"""
import ctypes as C
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "synth.c")
LIB_PATH = os.path.join(HERE, "libvbdr_synth.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-fPIC", "-shared", "-fopenmp",
           "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, d = C.c_void_p, C.c_uint32, C.c_uint64, C.c_double
        L.synth_create.restype = vp
        L.synth_create.argtypes = [u64, u32, d, u32, u64, u32, d, u32, d, d]
        L.synth_destroy.restype = None
        L.synth_destroy.argtypes = [vp]
        L.synth_hosts.restype = None
        L.synth_hosts.argtypes = [vp, vp, vp]
        L.synth_member.restype = u32
        L.synth_member.argtypes = [vp, u32, u64, u64]
        L.synth_slice.restype = u64
        L.synth_slice.argtypes = [vp, u64, vp, vp, vp]
        _lib = L
    return _lib


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    hosts: int
    zipf_s: float
    nmax: int
    pairs_per_slice: int
    slices: int
    m: int
    g: int
    k: int
    churn: int = 5
    copies_mean: float = 3.0
    n_heavy: int = 0
    heavy_lo: float = 1e6
    heavy_hi: float = 1e7

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


TINY = Workload("tiny", seed=0, hosts=1 << 12, zipf_s=1.1, nmax=10**4, pairs_per_slice=1 << 20,
                slices=12, m=1 << 18, g=256, k=4)
LINE_RATE = Workload("line_rate", seed=1, hosts=1 << 20, zipf_s=1.2, nmax=10**6,
                     pairs_per_slice=1 << 26, slices=64, m=1 << 26, g=1024, k=60)
MID = Workload("mid", seed=3, hosts=1 << 14, zipf_s=1.1, nmax=10**4, pairs_per_slice=1 << 22,
               slices=24, m=1 << 20, g=512, k=16)
STRESS = Workload("stress", seed=5, hosts=1 << 24, zipf_s=1.5, nmax=10**4, pairs_per_slice=1 << 27,
                  slices=144, m=1 << 24, g=2048, k=128, n_heavy=16)


def batched_workloads(seed: int = 4, n: int = 32):
    """Independent edge-router streams of uneven size: N_s = floor(2^U(16,24))
    pairs per slice, k in {4,...,128}, g in {128,...,1024}, pool 2^floor(U(16,25))
    clipped to 2^24, max(256, N_s/256) hosts with Zipf(1.1) opposite sets on
    1..10^4; 32 slices."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        N = int(2 ** rng.uniform(16, 24))
        k = int(rng.choice([4, 8, 16, 32, 64, 128]))
        g = int(rng.choice([128, 256, 512, 1024]))
        m = min(1 << int(rng.uniform(16, 25)), 1 << 24)
        out.append(Workload(f"batched{s}", seed=seed * 1000 + s, hosts=max(256, N // 256), zipf_s=1.1, nmax=10**4,
                            pairs_per_slice=N, slices=32, m=max(m, 2 * g), g=g, k=k))
    return out


class Stream:
    """A regenerable stream: ``slice(t)`` returns the N x 2 uint32 pairs of slice t."""

    def __init__(self, w: Workload):
        self.w = w
        self._h = _load().synth_create(w.seed, w.hosts, w.zipf_s, w.nmax, w.pairs_per_slice, w.churn,
                                       w.copies_mean, w.n_heavy, w.heavy_lo, w.heavy_hi)
        if not self._h:
            raise ValueError(f"bad workload {w}")
        self.aip = np.zeros(w.hosts, dtype=np.uint32)
        self.n = np.zeros(w.hosts, dtype=np.uint32)
        _load().synth_hosts(self._h, self.aip.ctypes.data, self.n.ctypes.data)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.synth_destroy(h)
            except Exception:
                pass
            self._h = None

    def slice(self, t: int, with_hidx: bool = False, host_pairs: np.ndarray = None, out: np.ndarray = None):
        N = self.w.pairs_per_slice
        pairs = out if out is not None else np.empty((N, 2), dtype=np.uint32)
        assert pairs.shape == (N, 2) and pairs.dtype == np.uint32 and pairs.flags.c_contiguous
        hidx = np.empty(N, dtype=np.uint32) if with_hidx else None
        if host_pairs is not None:
            assert host_pairs.shape == (self.w.hosts,) and host_pairs.dtype == np.uint32
        _load().synth_slice(self._h, t, pairs.ctypes.data, None if hidx is None else hidx.ctypes.data,
                            None if host_pairs is None else host_pairs.ctypes.data)
        return (pairs, hidx) if with_hidx else pairs

    def member(self, h: int, j: int, t: int) -> int:
        return int(_load().synth_member(self._h, h, j, t))


def exact_counts(slices_pairs, hosts) -> np.ndarray:
    """|OP(aip)| over the union of the given slices, for each aip in ``hosts``
    (Definition 1: distinct opposite hosts seen with aip in the window)."""
    hosts = np.asarray(hosts, dtype=np.uint32)
    if len(slices_pairs) == 0:
        return np.zeros(len(hosts), dtype=np.int64)
    allp = np.concatenate([np.asarray(p, dtype=np.uint32).reshape(-1, 2) for p in slices_pairs])
    key = (allp[:, 0].astype(np.uint64) << np.uint64(32)) | allp[:, 1].astype(np.uint64)
    uniq = np.unique(key)
    ua = (uniq >> np.uint64(32)).astype(np.uint32)
    vals, counts = np.unique(ua, return_counts=True)
    pos = np.searchsorted(vals, hosts)
    pos = np.clip(pos, 0, max(len(vals) - 1, 0))
    res = np.where((len(vals) > 0) & (vals[pos] == hosts), counts[pos], 0) if len(vals) else np.zeros(len(hosts))
    return res.astype(np.int64)
