"""Python binding of libvbdr.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; torch provides
device memory and the current HIP stream.  The library must be built
(``python -m paper_1810_13132_amd.build``); there is no fallback.

    sk = Sketch(m=1 << 18, g=256, k=4, hash_seed=0, layout="fast")
    sk.scan_slice(pairs)        # (n, 2) uint32/int32 CUDA tensor of (aip, bip)
    sk.advance_slice()
    est = sk.estimate(hosts)    # (h,) float32 CUDA tensor
"""
import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime libvbdr.so then binds to

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvbdr.so")

LAYOUTS = {"fast": 0, "small": 1, "packed": 2}
ESTIMATORS = {"hll": 0, "loglog": 1, "pcsa": 2}
NBINS = 33
STATUS = {0: "VBDR_OK", -1: "VBDR_EINVAL", -2: "VBDR_ENOMEM", -3: "VBDR_EHIP", -4: "VBDR_ESTATE"}


class VbdrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Info(C.Structure):
    _fields_ = [("m", C.c_uint64), ("g", C.c_uint32), ("b", C.c_uint32), ("L", C.c_uint32), ("k", C.c_uint32),
                ("layout", C.c_int32), ("A0", C.c_uint32), ("A1", C.c_uint32), ("t", C.c_uint64),
                ("state_bytes", C.c_uint64), ("est_parts", C.c_int32), ("scan_deferred", C.c_int32),
                ("Lc", C.c_uint32), ("dr_bits", C.c_uint32), ("est_tiled", C.c_int32),
                ("window_state_bytes", C.c_uint64), ("workspace_bytes", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [("scan_test_first", C.c_int32), ("scan_blocks_per_cu", C.c_uint32),
                ("est_blocks_per_cu", C.c_uint32), ("scan_binned", C.c_int32), ("est_binned", C.c_int32),
                ("est_parts", C.c_int32), ("est_bin_hosts", C.c_uint32),
                ("est_bin_cap", C.c_uint32), ("scan_defer", C.c_int32)]


class BatchParams(C.Structure):
    _fields_ = [("m", C.c_uint64), ("g", C.c_uint32), ("k", C.c_uint32), ("hash_seed", C.c_uint64),
                ("layout", C.c_int32)]


class BatchTuning(C.Structure):
    _fields_ = [("scan_tile", C.c_uint32), ("est_tile", C.c_uint32), ("blocks_per_cu", C.c_uint32),
                ("use_graph", C.c_int32)]


EXPORTS = ["vbdr_sketch_create", "vbdr_sketch_create_layout", "vbdr_sketch_create_packed", "vbdr_sketch_destroy",
           "vbdr_scan_slice",
           "vbdr_advance_slice", "vbdr_estimate", "vbdr_estimate_ex", "vbdr_sketch_info", "vbdr_export_state",
           "vbdr_import_state", "vbdr_last_error", "vbdr_sketch_set_tuning", "vbdr_sketch_get_tuning",
           "vbdr_mlp_create", "vbdr_mlp_destroy", "vbdr_features", "vbdr_estimate_learned", "vbdr_trainer_create",
           "vbdr_trainer_destroy", "vbdr_trainer_set_lr", "vbdr_trainer_step", "vbdr_trainer_grad",
           "vbdr_trainer_params", "vbdr_batch_create", "vbdr_batch_destroy", "vbdr_batch_sketch",
           "vbdr_batch_set_tuning", "vbdr_batch_get_tuning", "vbdr_batch_step", "vbdr_select_hosts",
           "vbdr_export_now", "vbdr_import_now", "vbdr_now_max", "vbdr_enable_pcsa", "vbdr_estimate_kind",
           "vbdr_export_pcsa", "vbdr_test_fail_alloc", "vbdr_estimate_noalloc",
           "vbdr_batch_set_mlp", "vbdr_mlp_set_plain_above"]
VOID_EXPORTS = ("vbdr_sketch_destroy", "vbdr_last_error", "vbdr_mlp_destroy", "vbdr_trainer_destroy",
                "vbdr_batch_destroy", "vbdr_batch_sketch")
MLP_IN, MLP_PARAMS = 67, 8577

_lib = None


def lib():
    """Load libvbdr.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1810_13132_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        L.vbdr_sketch_create.argtypes = [u64, u32, u32, u64, C.POINTER(vp)]
        L.vbdr_sketch_create_layout.argtypes = [u64, u32, u32, u64, i32, C.POINTER(vp)]
        L.vbdr_sketch_create_packed.argtypes = [u64, u32, u32, u64, u32, C.POINTER(vp)]
        L.vbdr_sketch_destroy.argtypes = [vp]
        L.vbdr_sketch_destroy.restype = None
        L.vbdr_scan_slice.argtypes = [vp, vp, u64, vp]
        L.vbdr_advance_slice.argtypes = [vp, vp]
        L.vbdr_estimate.argtypes = [vp, vp, u64, vp, vp]
        L.vbdr_estimate_ex.argtypes = [vp, vp, u64, vp, vp, vp, vp]
        L.vbdr_estimate_noalloc.argtypes = [vp, vp, u64, vp, vp]
        L.vbdr_sketch_info.argtypes = [vp, C.POINTER(Info)]
        L.vbdr_export_state.argtypes = [vp, vp, vp, vp, vp, vp]
        L.vbdr_import_state.argtypes = [vp, vp, vp, vp, vp, u64, vp]
        L.vbdr_sketch_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.vbdr_sketch_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.vbdr_mlp_create.argtypes = [vp, vp, vp, C.POINTER(vp)]
        L.vbdr_mlp_destroy.argtypes = [vp]
        L.vbdr_mlp_set_plain_above.argtypes = [vp, C.c_float]
        L.vbdr_features.argtypes = [vp, vp, u64, vp, vp]
        L.vbdr_estimate_learned.argtypes = [vp, vp, vp, u64, vp, vp, vp]
        L.vbdr_trainer_create.argtypes = [vp, C.c_float, C.POINTER(vp)]
        L.vbdr_trainer_destroy.argtypes = [vp]
        L.vbdr_trainer_set_lr.argtypes = [vp, C.c_float]
        L.vbdr_trainer_step.argtypes = [vp, vp, vp, u64, vp, vp]
        L.vbdr_trainer_grad.argtypes = [vp, vp, vp, u64, vp, vp, vp]
        L.vbdr_trainer_params.argtypes = [vp, vp, vp]
        L.vbdr_batch_create.argtypes = [u32, C.POINTER(BatchParams), C.POINTER(vp)]
        L.vbdr_batch_destroy.argtypes = [vp]
        L.vbdr_batch_sketch.argtypes = [vp, u32]
        L.vbdr_batch_set_tuning.argtypes = [vp, C.POINTER(BatchTuning)]
        L.vbdr_batch_set_mlp.argtypes = [vp, u32, vp]
        L.vbdr_batch_get_tuning.argtypes = [vp, C.POINTER(BatchTuning)]
        L.vbdr_select_hosts.argtypes = [vp, vp, u64, C.c_float, vp, vp, u64, vp, vp]
        L.vbdr_export_now.argtypes = [vp, vp, vp]
        L.vbdr_enable_pcsa.argtypes = [vp, i32]
        L.vbdr_estimate_kind.argtypes = [vp, vp, u64, i32, vp, vp, vp]
        L.vbdr_export_pcsa.argtypes = [vp, vp, vp]
        L.vbdr_import_now.argtypes = [vp, vp, vp]
        L.vbdr_now_max.argtypes = [vp, vp, vp, u64, vp]
        L.vbdr_batch_step.argtypes = [vp, C.POINTER(vp), C.POINTER(u64), C.POINTER(vp), C.POINTER(u64),
                                      C.POINTER(vp), vp]
        L.vbdr_test_fail_alloc.argtypes = [C.c_int64]
        L.vbdr_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name in VOID_EXPORTS:
                if name == "vbdr_batch_sketch":
                    L.vbdr_batch_sketch.restype = vp
                elif name != "vbdr_last_error":
                    getattr(L, name).restype = None
            else:
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise VbdrError(rc, lib().vbdr_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtypes, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


_U32 = (torch.int32, torch.uint32)


class Sketch:
    """A VBDR sketch living on the current device."""

    def __init__(self, m: int, g: int, k: int, hash_seed: int = 0, layout: str = "fast", Lc: int = 0, _borrow=None):
        """layout "fast", "small" or "packed" (z-bit DRs, Lc recorders per BDR; Lc = 0 means 33 - log2 g)."""
        self._owned = _borrow is None
        if _borrow is None:
            h = C.c_void_p()
            if layout == "packed":
                Lc = Lc or 33 - (int(g).bit_length() - 1)
                _check(lib().vbdr_sketch_create_packed(m, g, k, hash_seed, Lc, C.byref(h)))
            else:
                _check(lib().vbdr_sketch_create_layout(m, g, k, hash_seed, LAYOUTS[layout], C.byref(h)))
        else:
            h = C.c_void_p(_borrow)
        self._h = h
        i = self.info()
        self.layout = {v: key for key, v in LAYOUTS.items()}[i.layout]
        self.m, self.g, self.b, self.L, self.k = i.m, i.g, i.b, i.L, i.k
        self.A0, self.A1 = i.A0, i.A1
        self.Lc, self.dr_bits = i.Lc, i.dr_bits

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value and getattr(self, "_owned", True):
            lib().vbdr_sketch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Info:
        out = Info()
        _check(lib().vbdr_sketch_info(self._h, C.byref(out)))
        return out

    def set_tuning(self, scan_test_first: int = 0, scan_blocks_per_cu: int = 0, est_blocks_per_cu: int = 0,
                   scan_binned: int = 0, est_binned: int = 0, est_parts: int = 0, est_bin_hosts: int = 0,
                   est_bin_cap: int = 0, scan_defer: int = 0):
        t = Tuning(scan_test_first, scan_blocks_per_cu, est_blocks_per_cu, scan_binned, est_binned, est_parts,
                   est_bin_hosts, est_bin_cap, scan_defer)
        _check(lib().vbdr_sketch_set_tuning(self._h, C.byref(t)))

    def enable_pcsa(self, on: bool = True):
        """Keep PCSA runs from the next advance on (small layout)."""
        _check(lib().vbdr_enable_pcsa(self._h, 1 if on else 0))

    def estimate_kind(self, hosts: torch.Tensor, kind: str, with_raw: bool = False, stream=None):
        """Noise-removed estimates by `kind` in ("hll", "loglog", "pcsa")."""
        n = hosts.numel()
        out = torch.empty(n, dtype=torch.float32, device=hosts.device)
        raw = torch.empty(n, dtype=torch.float64, device=hosts.device) if with_raw else None
        if n:
            _check(lib().vbdr_estimate_kind(self._h, _dev_ptr(hosts, _U32, "hosts"), n, ESTIMATORS[kind],
                                            _dev_ptr(out, (torch.float32,), "out"),
                                            _dev_ptr(raw, (torch.float64,), "raw") if with_raw else None,
                                            _stream(stream)))
        return (out, raw) if with_raw else out

    def pcsa_registers(self, stream=None) -> np.ndarray:
        """(m,) PCSA runs of the last closed window (host copy)."""
        out = np.zeros(int(self.info().m), dtype=np.uint8)
        _check(lib().vbdr_export_pcsa(self._h, out.ctypes.data_as(C.c_void_p), _stream(stream)))
        return out

    def export_now(self, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """(m,) uint8 device map of the open slice's highest LBP1 per BDR (fast layout)."""
        m = int(self.info().m)
        if out is None:
            out = torch.empty(m, dtype=torch.uint8, device="cuda")
        _check(lib().vbdr_export_now(self._h, _dev_ptr(out, (torch.uint8,), "now"), _stream(stream)))
        return out

    def import_now(self, now: torch.Tensor, stream=None):
        """Make `now` ((m,) uint8 device) the open slice's LBP1 record (fast layout)."""
        if now.numel() != int(self.info().m):
            raise ValueError("now must hold m bytes")
        _check(lib().vbdr_import_now(self._h, _dev_ptr(now, (torch.uint8,), "now"), _stream(stream)))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().vbdr_sketch_get_tuning(self._h, C.byref(t)))
        return {"scan_test_first": t.scan_test_first, "scan_blocks_per_cu": t.scan_blocks_per_cu,
                "est_blocks_per_cu": t.est_blocks_per_cu, "scan_binned": t.scan_binned, "est_binned": t.est_binned,
                "est_parts": t.est_parts, "est_bin_hosts": t.est_bin_hosts,
                "est_bin_cap": t.est_bin_cap, "scan_defer": t.scan_defer}

    @property
    def t(self) -> int:
        return int(self.info().t)

    def scan_slice(self, pairs: torch.Tensor, stream=None):
        n = pairs.numel() // 2
        if pairs.numel() != 2 * n:
            raise ValueError("pairs must hold an even number of uint32")
        ptr = _dev_ptr(pairs, _U32, "pairs") if n else C.c_void_p()
        _check(lib().vbdr_scan_slice(self._h, ptr, n, _stream(stream)))

    def advance_slice(self, stream=None):
        _check(lib().vbdr_advance_slice(self._h, _stream(stream)))

    def estimate(self, hosts: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        n = hosts.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=hosts.device)
        if n:
            _check(lib().vbdr_estimate(self._h, _dev_ptr(hosts, _U32, "hosts"), n,
                                       _dev_ptr(out, (torch.float32,), "out"), _stream(stream)))
        return out

    def estimate_noalloc(self, hosts: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """vbdr_estimate with the library's static scratch instead of the sketch's
        workspaces; out (n float32, device) is the caller's."""
        n = hosts.numel()
        if out.numel() != n:
            raise ValueError("out must hold one float per host")
        if n:
            _check(lib().vbdr_estimate_noalloc(self._h, _dev_ptr(hosts, _U32, "hosts"), n,
                                               _dev_ptr(out, (torch.float32,), "out"), _stream(stream)))
        return out

    def estimate_ex(self, hosts: torch.Tensor, stream=None):
        """(estimate float32, raw E_s float64, register histogram (n, 33) int32)."""
        n = hosts.numel()
        out = torch.empty(n, dtype=torch.float32, device=hosts.device)
        raw = torch.empty(n, dtype=torch.float64, device=hosts.device)
        hist = torch.empty((n, NBINS), dtype=torch.int32, device=hosts.device)
        if n:
            _check(lib().vbdr_estimate_ex(self._h, _dev_ptr(hosts, _U32, "hosts"), n,
                                          _dev_ptr(out, (torch.float32,), "out"),
                                          _dev_ptr(raw, (torch.float64,), "raw"),
                                          _dev_ptr(hist, (torch.int32,), "hist"), _stream(stream)))
        return out, raw, hist

    def features(self, hosts: torch.Tensor, stream=None) -> torch.Tensor:
        """(n, 67) float32 features of the learned estimator for these hosts."""
        n = hosts.numel()
        feats = torch.empty((n, MLP_IN), dtype=torch.float32, device=hosts.device)
        if n:
            _check(lib().vbdr_features(self._h, _dev_ptr(hosts, _U32, "hosts"), n,
                                       _dev_ptr(feats, (torch.float32,), "feats"), _stream(stream)))
        return feats

    def estimate_learned(self, mlp: "MLP", hosts: torch.Tensor, out: torch.Tensor = None, with_fallback=False,
                         stream=None):
        n = hosts.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=hosts.device)
        fb = torch.empty(n, dtype=torch.uint8, device=hosts.device) if with_fallback else None
        if n:
            _check(lib().vbdr_estimate_learned(self._h, mlp._h, _dev_ptr(hosts, _U32, "hosts"), n,
                                               _dev_ptr(out, (torch.float32,), "out"),
                                               None if fb is None else _dev_ptr(fb, (torch.uint8,), "fallback"),
                                               _stream(stream)))
        return (out, fb) if with_fallback else out

    def state(self, stream=None) -> dict:
        """Canonical state as numpy arrays: dr (m, L) uint8, bs (m,) uint32, reg (m,) uint8, hist (33,) uint64."""
        m, L = self.m, self.L
        dr = np.empty((m, L), dtype=np.uint8)
        bs = np.empty(m, dtype=np.uint32)
        reg = np.empty(m, dtype=np.uint8)
        hist = np.empty(NBINS, dtype=np.uint64)
        _check(lib().vbdr_export_state(self._h, dr.ctypes.data, bs.ctypes.data, reg.ctypes.data, hist.ctypes.data,
                                       _stream(stream)))
        return {"dr": dr, "bs": bs, "reg": reg, "hist": hist, "t": self.t}

    def registers(self, stream=None):
        """(reg (m,) uint8, hist (33,) uint64) of the last closed window, without the DRs."""
        reg = np.empty(self.m, dtype=np.uint8)
        hist = np.empty(NBINS, dtype=np.uint64)
        _check(lib().vbdr_export_state(self._h, None, None, reg.ctypes.data, hist.ctypes.data, _stream(stream)))
        return reg, hist

    def load_state(self, state: dict, stream=None):
        dr = np.ascontiguousarray(state["dr"], dtype=np.uint8)
        reg = np.ascontiguousarray(state["reg"], dtype=np.uint8)
        hist = np.ascontiguousarray(state["hist"], dtype=np.uint64)
        bs = state.get("bs")
        bs = None if bs is None else np.ascontiguousarray(bs, dtype=np.uint32)
        if dr.shape != (self.m, self.L) or reg.shape != (self.m,) or hist.shape != (NBINS,):
            raise ValueError("state shapes do not match the sketch")
        _check(lib().vbdr_import_state(self._h, dr.ctypes.data, None if bs is None else bs.ctypes.data,
                                       reg.ctypes.data, hist.ctypes.data, int(state["t"]), _stream(stream)))


def now_max(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Element-wise MAX of two uint8 device maps (the exchange's reduction)."""
    if a.numel() != b.numel():
        raise ValueError("maps differ in length")
    out = torch.empty_like(a) if out is None else out
    _check(lib().vbdr_now_max(_dev_ptr(a, (torch.uint8,), "a"), _dev_ptr(b, (torch.uint8,), "b"),
                              _dev_ptr(out, (torch.uint8,), "out"), a.numel(), _stream(stream)))
    return out


def select_hosts(est: torch.Tensor, hosts: torch.Tensor, threshold: float, cap: int = None, stream=None):
    """Super points: the hosts whose estimate is at least `threshold`.
    Returns (hosts, estimates, count) with hosts/estimates on the device in
    unspecified order; count is the number selected (only min(count, cap)
    are returned)."""
    n = est.numel()
    if hosts.numel() != n:
        raise ValueError("est and hosts must have the same length")
    cap = n if cap is None else cap
    oh = torch.empty(max(cap, 1), dtype=torch.int32, device=est.device)
    oe = torch.empty(max(cap, 1), dtype=torch.float32, device=est.device)
    cnt = torch.empty(1, dtype=torch.int32, device=est.device)
    _check(lib().vbdr_select_hosts(_dev_ptr(est, (torch.float32,), "est") if n else None,
                                   _dev_ptr(hosts, _U32, "hosts") if n else None, n, float(threshold),
                                   _dev_ptr(oh, _U32, "out_hosts"), _dev_ptr(oe, (torch.float32,), "out_est"), cap,
                                   _dev_ptr(cnt, _U32, "count"), _stream(stream)))
    c = int(cnt.item())
    k = min(c, cap)
    return oh[:k], oe[:k], c


def fail_allocation_after(n: int):
    """Testing aid: the library's device allocation after n more successful
    ones fails (VBDR_ENOMEM); n < 0 cancels."""
    _check(lib().vbdr_test_fail_alloc(int(n)))


def to_device_u32(a: np.ndarray, device="cuda") -> torch.Tensor:
    """Copy a uint32 numpy array to the device (as int32 storage, same bits)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def _host_f32(a, n, name):
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.shape != (n,):
        raise ValueError(f"{name} must hold {n} floats")
    return a


class MLP:
    """A learned-estimator network on the current device (bf16 weights)."""

    def __init__(self, params, env_lo=None, env_hi=None, plain_above=None):
        p = _host_f32(params, MLP_PARAMS, "params")
        lo = None if env_lo is None else _host_f32(env_lo, MLP_IN, "env_lo")
        hi = None if env_hi is None else _host_f32(env_hi, MLP_IN, "env_hi")
        h = C.c_void_p()
        _check(lib().vbdr_mlp_create(p.ctypes.data, None if lo is None else lo.ctypes.data,
                                     None if hi is None else hi.ctypes.data, C.byref(h)))
        self._h = h
        if plain_above is not None:
            self.set_plain_above(plain_above)

    def set_plain_above(self, threshold: float):
        """Keep the plain estimate where it is at least `threshold` (inf: never)."""
        _check(lib().vbdr_mlp_set_plain_above(self._h, float(threshold)))

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value:
            lib().vbdr_mlp_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trainer:
    """Float32 Adam training of the learned estimator on the current device."""

    def __init__(self, params, lr: float = 1e-3):
        p = _host_f32(params, MLP_PARAMS, "params")
        h = C.c_void_p()
        _check(lib().vbdr_trainer_create(p.ctypes.data, lr, C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value:
            lib().vbdr_trainer_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_lr(self, lr: float):
        _check(lib().vbdr_trainer_set_lr(self._h, lr))

    def step(self, feats: torch.Tensor, targets: torch.Tensor, loss: torch.Tensor = None, stream=None):
        n = targets.numel()
        _check(lib().vbdr_trainer_step(self._h, _dev_ptr(feats, (torch.float32,), "feats"),
                                       _dev_ptr(targets, (torch.float32,), "targets"), n,
                                       None if loss is None else _dev_ptr(loss, (torch.float32,), "loss"),
                                       _stream(stream)))

    def grad(self, feats: torch.Tensor, targets: torch.Tensor, stream=None):
        n = targets.numel()
        g = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.zeros(1, dtype=torch.float32, device=feats.device)
        _check(lib().vbdr_trainer_grad(self._h, _dev_ptr(feats, (torch.float32,), "feats"),
                                       _dev_ptr(targets, (torch.float32,), "targets"), n,
                                       _dev_ptr(g, (torch.float32,), "grads"),
                                       _dev_ptr(loss, (torch.float32,), "loss"), _stream(stream)))
        return g, loss

    def params(self, stream=None) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().vbdr_trainer_params(self._h, out.ctypes.data, _stream(stream)))
        return out


class Batch:
    """Independent sketches stepped together (persistent kernels, graph replay).

    params: list of dicts with m, g, k, hash_seed and layout ("fast"/"small")."""

    def __init__(self, params):
        arr = (BatchParams * len(params))()
        for i, p in enumerate(params):
            arr[i] = BatchParams(p["m"], p["g"], p["k"], p.get("hash_seed", 0), LAYOUTS[p.get("layout", "fast")])
        h = C.c_void_p()
        _check(lib().vbdr_batch_create(len(params), arr, C.byref(h)))
        self._h = h
        self.n = len(params)
        self.sketches = [Sketch(0, 0, 0, _borrow=lib().vbdr_batch_sketch(h, i)) for i in range(self.n)]

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value:
            for s in getattr(self, "sketches", []):
                s._h = None
            lib().vbdr_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, scan_tile=8192, est_tile=64, blocks_per_cu=8, use_graph=True):
        t = BatchTuning(scan_tile, est_tile, blocks_per_cu, 1 if use_graph else 0)
        _check(lib().vbdr_batch_set_tuning(self._h, C.byref(t)))

    def set_mlp(self, i: int, mlp: "MLP" = None):
        """Learned estimates for sketch i (None: plain); keep `mlp` alive while steps use it."""
        _check(lib().vbdr_batch_set_mlp(self._h, i, None if mlp is None else mlp._h))

    def get_tuning(self) -> dict:
        t = BatchTuning()
        _check(lib().vbdr_batch_get_tuning(self._h, C.byref(t)))
        return {"scan_tile": t.scan_tile, "est_tile": t.est_tile, "blocks_per_cu": t.blocks_per_cu,
                "use_graph": bool(t.use_graph)}

    def step(self, pairs, hosts, outs, stream=None):
        """pairs, hosts, outs: lists (one per sketch) of device tensors."""
        n = self.n
        if not (len(pairs) == len(hosts) == len(outs) == n):
            raise ValueError("one pairs, hosts and out tensor per sketch")
        P, NP, Hh, NH, O = (C.c_void_p * n)(), (C.c_uint64 * n)(), (C.c_void_p * n)(), (C.c_uint64 * n)(), \
            (C.c_void_p * n)()
        for i in range(n):
            npairs = pairs[i].numel() // 2
            P[i] = _dev_ptr(pairs[i], _U32, "pairs").value if npairs else None
            NP[i] = npairs
            nh = hosts[i].numel()
            if outs[i].numel() != nh:
                raise ValueError("out must have one float per host")
            Hh[i] = _dev_ptr(hosts[i], _U32, "hosts").value if nh else None
            O[i] = _dev_ptr(outs[i], (torch.float32,), "out").value if nh else None
            NH[i] = nh
        _check(lib().vbdr_batch_step(self._h, P, NP, Hh, NH, O, _stream(stream)))
