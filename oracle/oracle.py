"""ctypes view of the CPU oracle -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads oracle/liboracle_vbdr.so (plain C, no HIP) and wraps
it with numpy arrays.  See vbdr_oracle.c for the paper passages followed and
the readings taken.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_vbdr.so")

SERIAL, GFAST, GSMALL, GPACKED = 0, 1, 2, 3
HLL, LOGLOG, PCSA = 0, 1, 2  # estimators over the pool
NBINS = 33

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle.build import build_oracle
            build_oracle()
        L = C.CDLL(LIB_PATH)
        u32, u64, vp = C.c_uint32, C.c_uint64, C.c_void_p
        L.vbdro_murmur3_32.restype = u32
        L.vbdro_murmur3_32.argtypes = [vp, u64, u32]
        L.vbdro_H.restype = u32
        L.vbdro_H.argtypes = [u32, u64, u32]
        L.vbdro_splitmix64.restype = u64
        L.vbdro_splitmix64.argtypes = [vp]
        L.vbdro_lbp1.restype = u32
        L.vbdro_lbp1.argtypes = [u32, u32]
        L.vbdro_create.restype = vp
        L.vbdro_create.argtypes = [u64, u32, u32, u64, C.c_int]
        L.vbdro_create_packed.restype = vp
        L.vbdro_create_packed.argtypes = [u64, u32, u32, u64, u32]
        L.vbdro_destroy.restype = None
        L.vbdro_destroy.argtypes = [vp]
        L.vbdro_phy_idx.restype = u32
        L.vbdro_phy_idx.argtypes = [vp, u32, u32]
        L.vbdro_pair_map.restype = None
        L.vbdro_pair_map.argtypes = [vp, vp, u64, vp, vp]
        L.vbdro_map_pairs.restype = C.c_int
        L.vbdro_map_pairs.argtypes = [u64, u32, u64, vp, u64, vp, vp]
        L.vbdro_scan.restype = None
        L.vbdro_scan.argtypes = [vp, vp, u64]
        L.vbdro_advance.restype = None
        L.vbdro_advance.argtypes = [vp]
        L.vbdro_alpha.restype = C.c_double
        L.vbdro_alpha.argtypes = [C.c_double]
        L.vbdro_hll_from_hist.restype = C.c_double
        L.vbdro_hll_from_hist.argtypes = [vp, C.c_double]
        L.vbdro_estimate.restype = None
        L.vbdro_estimate.argtypes = [vp, vp, u64, vp, vp, vp]
        L.vbdro_estimate_registers.restype = C.c_int
        L.vbdro_estimate_registers.argtypes = [u64, u32, u64, vp, vp, u64, vp, vp, vp]
        L.vbdro_replay_state.restype = None
        L.vbdro_replay_state.argtypes = [vp, u64, u32, u32, u32, u32, u32, vp, vp]
        L.vbdro_sum_lbp1.restype = u64
        L.vbdro_sum_lbp1.argtypes = [vp, u32]
        L.vbdro_loglog_alpha.restype = C.c_double
        L.vbdro_loglog_alpha.argtypes = [C.c_double]
        L.vbdro_estimate_kind.restype = C.c_int
        L.vbdro_estimate_kind.argtypes = [vp, vp, u64, C.c_int, vp, vp]
        L.vbdro_get_preg.restype = C.c_int
        L.vbdro_get_preg.argtypes = [vp, vp]
        L.vbdro_params.restype = None
        L.vbdro_params.argtypes = [vp, vp]
        L.vbdro_get_state.restype = None
        L.vbdro_get_state.argtypes = [vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def murmur3_32(data: bytes, seed: int) -> int:
    buf = np.frombuffer(data, dtype=np.uint8) if len(data) else np.zeros(1, np.uint8)
    return int(lib().vbdro_murmur3_32(_ptr(buf), len(data), seed & 0xFFFFFFFF))


def H(x: int, N: int, A: int) -> int:
    return int(lib().vbdro_H(x & 0xFFFFFFFF, N, A & 0xFFFFFFFF))


def splitmix64(state: int):
    s = np.array([state], dtype=np.uint64)
    out = int(lib().vbdro_splitmix64(_ptr(s)))
    return out, int(s[0])


def lbp1(w: int, b: int) -> int:
    return int(lib().vbdro_lbp1(w & 0xFFFFFFFF, b))


def alpha(q: float) -> float:
    return float(lib().vbdro_alpha(q))


def loglog_alpha(q: float) -> float:
    return float(lib().vbdro_loglog_alpha(float(q)))


def hll_from_hist(hist, q: float) -> float:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    assert h.shape == (NBINS,)
    return float(lib().vbdro_hll_from_hist(_ptr(h), float(q)))


def map_pairs(m: int, g: int, hash_seed: int, pairs: np.ndarray):
    """(pidx, LBP1) of each pair for a pool of m BDRs, without building the pool."""
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    pidx = np.zeros(n, dtype=np.uint32)
    rho = np.zeros(n, dtype=np.uint8)
    if lib().vbdro_map_pairs(m, g, hash_seed, _ptr(pairs), n, _ptr(pidx), _ptr(rho)) != 0:
        raise ValueError("bad parameters")
    return pidx, rho


def estimate_registers(m: int, g: int, hash_seed: int, reg: np.ndarray, hosts, with_raw: bool = False,
                       with_hist: bool = False):
    """The estimate of Alg. 5 (histogram, HyperLogLog, noise removal) over a
    register array reg (m uint8) given by the caller instead of a sketch's."""
    reg = np.ascontiguousarray(reg, dtype=np.uint8).reshape(-1)
    assert reg.shape == (m,)
    hosts = np.ascontiguousarray(hosts, dtype=np.uint32).reshape(-1)
    n = hosts.shape[0]
    out = np.zeros(n, dtype=np.float32)
    raw = np.zeros(n, dtype=np.float64)
    hist = np.zeros((n, NBINS), dtype=np.uint32) if with_hist else None
    if lib().vbdro_estimate_registers(m, g, hash_seed, _ptr(reg), _ptr(hosts), n, _ptr(out), _ptr(raw),
                                      _ptr(hist)) != 0:
        raise ValueError("bad parameters or register values")
    res = [out]
    if with_raw:
        res.append(raw)
    if with_hist:
        res.append(hist)
    return res[0] if len(res) == 1 else tuple(res)


class Sketch:
    """One VBDR sketch held by the oracle."""

    def __init__(self, m: int, g: int, k: int, hash_seed: int, layout: int = GFAST, Lc: int = 0):
        if layout == GPACKED:
            self._h = lib().vbdro_create_packed(m, g, k, hash_seed, Lc)
        else:
            self._h = lib().vbdro_create(m, g, k, hash_seed, layout)
        if not self._h:
            raise ValueError(f"oracle rejects m={m} g={g} k={k} layout={layout} Lc={Lc}")
        p = self.params()
        self.m, self.g, self.b, self.L, self.k = p[0], p[1], p[2], p[3], p[4]
        self.layout, self.A0, self.A1 = p[5], p[6], p[7]
        self.Lc, self.sat = p[9], p[10]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().vbdro_destroy(h)
            self._h = None

    def params(self):
        out = np.zeros(11, dtype=np.uint64)
        lib().vbdro_params(self._h, _ptr(out))
        return [int(v) for v in out]

    @property
    def t(self) -> int:
        return self.params()[8]

    def phy_idx(self, aip: int, i: int) -> int:
        return int(lib().vbdro_phy_idx(self._h, aip, i))

    def pair_map(self, pairs: np.ndarray):
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        n = pairs.shape[0]
        pidx = np.zeros(n, dtype=np.uint32)
        rho = np.zeros(n, dtype=np.uint8)
        if n:
            lib().vbdro_pair_map(self._h, _ptr(pairs), n, _ptr(pidx), _ptr(rho))
        return pidx, rho

    def scan(self, pairs: np.ndarray):
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        if pairs.shape[0]:
            lib().vbdro_scan(self._h, _ptr(pairs), pairs.shape[0])

    def advance(self):
        lib().vbdro_advance(self._h)

    def estimate(self, hosts, with_raw: bool = False, with_hist: bool = False):
        hosts = np.ascontiguousarray(hosts, dtype=np.uint32).reshape(-1)
        n = hosts.shape[0]
        out = np.zeros(n, dtype=np.float32)
        raw = np.zeros(n, dtype=np.float64) if with_raw else None
        hist = np.zeros((n, NBINS), dtype=np.uint32) if with_hist else None
        if n:
            lib().vbdro_estimate(self._h, _ptr(hosts), n, _ptr(out), _ptr(raw), _ptr(hist))
        res = [out]
        if with_raw:
            res.append(raw)
        if with_hist:
            res.append(hist)
        return res[0] if len(res) == 1 else tuple(res)

    def sum_lbp1(self, aip: int) -> int:
        return int(lib().vbdro_sum_lbp1(self._h, aip))

    def estimate_kind(self, hosts, kind: int, with_raw: bool = False):
        """Noise-removed LogLog (kind LOGLOG) or PCSA (kind PCSA, small layout) estimates."""
        if kind == HLL:
            return self.estimate(hosts, with_raw=with_raw)
        hosts = np.ascontiguousarray(hosts, dtype=np.uint32).reshape(-1)
        n = hosts.shape[0]
        out = np.zeros(n, dtype=np.float32)
        raw = np.zeros(n, dtype=np.float64)
        if lib().vbdro_estimate_kind(self._h, _ptr(hosts), n, kind, _ptr(out), _ptr(raw)) != 0:
            raise ValueError("estimator not available for this sketch")
        return (out, raw) if with_raw else out

    def pcsa_registers(self):
        """(m,) PCSA runs of the last closed window (small and packed layouts)."""
        out = np.zeros(self.m, dtype=np.uint8)
        if lib().vbdro_get_preg(self._h, _ptr(out)) != 0:
            raise ValueError("PCSA registers need the small layout")
        return out

    def state(self):
        """Canonical state: dict of dr (m, L), bs (m,), now (m,), reg (m,), hist (33,)."""
        m, L = self.m, self.L
        dr = np.zeros((m, L), dtype=np.uint8)
        bs = np.zeros(m, dtype=np.uint32)
        now = np.zeros(m, dtype=np.uint8)
        reg = np.zeros(m, dtype=np.uint8)
        hist = np.zeros(NBINS, dtype=np.uint64)
        lib().vbdro_get_state(self._h, _ptr(dr), _ptr(bs), _ptr(now), _ptr(reg), _ptr(hist))
        return {"dr": dr, "bs": bs, "now": now, "reg": reg, "hist": hist, "t": self.t}


def select_hosts(est, hosts, threshold: float):
    """Super points over the window (Sec. 1 and Sec. 2.3 motivate per-host
    cardinalities for superspreader detection): every host whose estimate is
    at least the threshold, as a sorted array of (host, estimate) rows.  The
    definition written out; NaN compares false and is never selected."""
    est = np.asarray(est, dtype=np.float32).reshape(-1)
    hosts = np.asarray(hosts, dtype=np.uint32).reshape(-1)
    keep = [i for i in range(len(est)) if est[i] >= np.float32(threshold)]
    rows = sorted((int(hosts[i]), float(est[i])) for i in keep)
    return rows
