"""Thin ctypes binding of libpolymul.so (include/polymul.h).

Argument marshalling only: device memory comes from torch tensors on the
current HIP device, streams from torch.cuda.Stream; every step of the product
runs in the library's kernels.  Raises if the HIP library is not built: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolymul.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "polymul.h")

PM_OK, PM_EINVAL, PM_EUNSORTED, PM_EOVERFLOW, PM_ERANGE, PM_ECAPACITY, PM_ENOMEM, PM_EDEVICE, PM_EBUSY = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
RING_CODE = {"modp": 0, "f64": 1, "i64": 2, "modq": 3, "z192": 4}


class pm_layout(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_uint32), ("bits", ctypes.c_uint32), ("ring", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class pm_cpoly(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("keys", ctypes.c_void_p), ("coefs", ctypes.c_void_p)]


class pm_poly(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("n_out", ctypes.c_void_p), ("keys", ctypes.c_void_p),
                ("coefs", ctypes.c_void_p)]


class PolymulError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = lib().pm_strerror(code).decode()
        if code == PM_EDEVICE:
            msg += ": " + lib().pm_last_error().decode()
        super().__init__(f"{where}: {msg} ({code})" if where else f"{msg} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libpolymul.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(python -m paper_1303_7425_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i64p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        L.pm_mul_bound.argtypes = [ctypes.POINTER(pm_layout), ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_cpoly),
                                   i64p, i64p, vp]
        L.pm_mul.argtypes = [ctypes.POINTER(pm_layout), ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_cpoly),
                             ctypes.POINTER(pm_poly), vp, i64, vp]
        L.pm_mul_batch_bound.argtypes = [ctypes.POINTER(pm_layout), i64, ctypes.POINTER(pm_cpoly),
                                         ctypes.POINTER(pm_cpoly), i64p, i64p, vp]
        L.pm_mul_batch.argtypes = [ctypes.POINTER(pm_layout), i64, ctypes.POINTER(pm_cpoly),
                                   ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_poly), vp, i64, vp]
        L.pm_plan_from_stats.argtypes = [ctypes.POINTER(pm_layout), i64, i64p, i64p,
                                         ctypes.POINTER(ctypes.c_uint64), i64p, i64p]
        L.pm_set_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.pm_last_call_status.argtypes = [vp]
        L.pm_last_call_info.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), i64p]
        L.pm_profile_enable.argtypes = [ctypes.c_int32]
        L.pm_profile_read.argtypes = [ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_double), i64p]
        L.pm_strerror.restype = ctypes.c_char_p
        L.pm_strerror.argtypes = [ctypes.c_int]
        L.pm_last_error.restype = ctypes.c_char_p
        L.pm_version.restype = ctypes.c_char_p
        L.pm_batch_prepare.argtypes = [ctypes.POINTER(pm_layout), i64, ctypes.POINTER(pm_cpoly),
                                       ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_poly), vp, i64, vp,
                                       ctypes.POINTER(vp)]
        L.pm_batch_launch.argtypes = [vp, vp]
        L.pm_batch_destroy.argtypes = [vp]
        L.pm_autotune.argtypes = [ctypes.POINTER(pm_layout), ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_cpoly),
                                  ctypes.POINTER(pm_poly), vp, i64, vp, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.pm_set_radix.argtypes = [ctypes.c_int32]
        L.pm_mul_noalloc.argtypes = [ctypes.POINTER(pm_layout), ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_cpoly),
                                     ctypes.POINTER(pm_poly), vp]
        L.pm_mul_batch_drain.argtypes = [ctypes.POINTER(pm_layout), i64, ctypes.POINTER(pm_cpoly),
                                         ctypes.POINTER(pm_cpoly), vp, i64, vp, i64, DRAIN_FN, vp, vp, i64p]
        L.pm_dense_ceiling.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp]
        L.pm_autotune_save.argtypes = [ctypes.c_char_p]
        L.pm_autotune_load.argtypes = [ctypes.c_char_p]
        L.pm_ival_grid.argtypes = [i64, i64, ctypes.c_int32, i64p, i64p]
        L.pm_ival_splitters.argtypes = [ctypes.POINTER(ctypes.c_uint64), i64, ctypes.POINTER(ctypes.c_uint64), i64,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), i64p]
        if hasattr(L, "pm_server_create"):
            L.pm_server_create.restype = vp
            L.pm_server_create.argtypes = [i64, ctypes.c_int32]
            L.pm_server_submit.argtypes = [vp, ctypes.POINTER(pm_layout), ctypes.POINTER(pm_cpoly),
                                           ctypes.POINTER(pm_cpoly), ctypes.POINTER(pm_poly),
                                           ctypes.POINTER(ctypes.c_uint64)]
            L.pm_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]
            L.pm_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
            L.pm_server_latencies.restype = i64
            L.pm_server_latencies.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64]
            L.pm_server_latency.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
            L.pm_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/polymul.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text)))


def make_layout(nvars: int, bits: int, ring: str) -> pm_layout:
    return pm_layout(nvars, bits, RING_CODE[ring], 0)


def _check(rc: int, where: str):
    if rc != PM_OK:
        raise PolymulError(rc, where)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------
# device-resident polynomials
# ----------------------------------------------------------------------------
@dataclass
class DevPoly:
    """Term arrays on the GPU: keys int64 (u64 bits), coefs int64 / float64
    (z192: an (n, 3) int64 array of two's-complement words)."""
    keys: object
    coefs: object
    n: int

    def numpy(self):
        k = self.keys[: self.n].cpu().numpy().view(np.uint64)
        c = self.coefs[: self.n].cpu().numpy()
        if c.dtype == np.int64 and self.coef_kind in ("modp", "modq", "z192"):
            c = c.view(np.uint64)
        return k, c

    coef_kind: str = "modp"


def to_device(poly, device="cuda"):
    """workloads.Poly -> DevPoly (keys and coefficient bits copied to HBM)."""
    import torch
    ring = poly.layout.ring
    k = torch.from_numpy(np.ascontiguousarray(poly.keys).view(np.int64)).to(device)
    if ring == "f64":
        c = torch.from_numpy(np.ascontiguousarray(poly.coefs, dtype=np.float64)).to(device)
    else:
        c = torch.from_numpy(np.ascontiguousarray(poly.coefs).view(np.int64)).to(device)
    return DevPoly(k, c, len(poly), ring)


def _cpoly(p: DevPoly) -> pm_cpoly:
    return pm_cpoly(p.n, p.keys.data_ptr() if p.n else None, p.coefs.data_ptr() if p.n else None)


class Workspace:
    """A growable device byte buffer reused across calls."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
        return self.buf


def bound(layout, f: DevPoly, g: DevPoly, stream=None):
    L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
    mt, wb = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().pm_mul_bound(ctypes.byref(L), ctypes.byref(_cpoly(f)), ctypes.byref(_cpoly(g)),
                              ctypes.byref(mt), ctypes.byref(wb), _stream_ptr(stream)), "pm_mul_bound")
    return int(mt.value), int(wb.value)


def alloc_out(cap: int, ring: str):
    import torch
    k = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
    shape = (max(cap, 1), 3) if ring == "z192" else (max(cap, 1),)
    c = torch.empty(shape, dtype=torch.float64 if ring == "f64" else torch.int64, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    return k, c, n


def mul(layout, f: DevPoly, g: DevPoly, out=None, workspace: Workspace | None = None, stream=None,
        sync: bool = True):
    """h = f * g on the GPU.  Returns DevPoly (n read back when sync=True)."""
    import torch
    L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
    ring = {v: k for k, v in RING_CODE.items()}[L.ring]
    cap, wbytes = bound(L, f, g, stream)
    if out is None:
        out = alloc_out(cap, ring)
    hk, hc, hn = out
    ws = (workspace or Workspace()).get(wbytes)
    h = pm_poly(min(hk.numel(), hc.numel()), hn.data_ptr(), hk.data_ptr(), hc.data_ptr())
    _check(lib().pm_mul(ctypes.byref(L), ctypes.byref(_cpoly(f)), ctypes.byref(_cpoly(g)), ctypes.byref(h),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)), "pm_mul")
    n = -1
    if sync:
        (stream or torch.cuda.current_stream()).synchronize()
        n = int(hn.item())
    return DevPoly(hk, hc, n, ring)


NOALLOC_SCRATCH_BYTES = 64 << 20


def mul_noalloc(layout, f: DevPoly, g: DevPoly, out, stream=None, sync: bool = True):
    """h = f * g through pm_mul_noalloc: the library uses its static device
    scratch, so only the caller's output arrays `out` = (keys, coefs, n) are
    passed.  Returns DevPoly (n read back when sync=True)."""
    import torch
    L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
    ring = {v: k for k, v in RING_CODE.items()}[L.ring]
    hk, hc, hn = out
    h = pm_poly(min(hk.numel(), hc.numel()), hn.data_ptr(), hk.data_ptr(), hc.data_ptr())
    _check(lib().pm_mul_noalloc(ctypes.byref(L), ctypes.byref(_cpoly(f)), ctypes.byref(_cpoly(g)), ctypes.byref(h),
                                _stream_ptr(stream)), "pm_mul_noalloc")
    n = -1
    if sync:
        (stream or torch.cuda.current_stream()).synchronize()
        n = int(hn.item())
    return DevPoly(hk, hc, n, ring)


class MulCall:
    """A prepared pm_mul call: bound, output arrays and workspace allocated once;
    `run()` enqueues the product (validation included) on the stream."""

    def __init__(self, layout, f: DevPoly, g: DevPoly, workspace: Workspace | None = None, stream=None,
                 capacity: int | None = None):
        self.L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
        self.ring = {v: k for k, v in RING_CODE.items()}[self.L.ring]
        self.f, self.g, self.stream = f, g, stream
        self.cf, self.cg = _cpoly(f), _cpoly(g)
        self.cap, self.ws_bytes = bound(self.L, f, g, stream)
        if capacity is not None:  # a known result size below the bound (results past it are not written)
            self.cap = min(self.cap, int(capacity))
        self.out = alloc_out(self.cap, self.ring)
        hk, hc, hn = self.out
        self.h = pm_poly(self.cap, hn.data_ptr(), hk.data_ptr(), hc.data_ptr())
        self.ws = (workspace or Workspace()).get(self.ws_bytes)
        self.sp = _stream_ptr(stream)

    def run(self):
        _check(lib().pm_mul(ctypes.byref(self.L), ctypes.byref(self.cf), ctypes.byref(self.cg),
                            ctypes.byref(self.h), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), self.sp),
               "pm_mul")

    def n(self) -> int:
        return int(self.out[2].item())

    def result(self) -> DevPoly:
        return DevPoly(self.out[0], self.out[1], self.n(), self.ring)


class BatchCall:
    """A prepared pm_mul_batch call: bound, outputs and workspace allocated once,
    then `run()` enqueues the batch (re-validating the operands each time)."""

    def __init__(self, layout, fs, gs, workspace: Workspace | None = None, stream=None):
        import torch
        self.L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
        self.ring = {v: k for k, v in RING_CODE.items()}[self.L.ring]
        self.count = len(fs)
        self.fs, self.gs = fs, gs
        self.cf = (pm_cpoly * self.count)(*[_cpoly(p) for p in fs])
        self.cg = (pm_cpoly * self.count)(*[_cpoly(p) for p in gs])
        mt = (ctypes.c_int64 * self.count)()
        wb = ctypes.c_int64(0)
        self.stream = stream
        _check(lib().pm_mul_batch_bound(ctypes.byref(self.L), self.count, self.cf, self.cg, mt, ctypes.byref(wb),
                                        _stream_ptr(stream)), "pm_mul_batch_bound")
        self.bounds = [int(x) for x in mt]
        self.ws_bytes = int(wb.value)
        tot = sum(max(b, 1) for b in self.bounds)
        self.out_k = torch.empty(tot, dtype=torch.int64, device="cuda")
        self.out_c = torch.empty(tot, dtype=torch.float64 if self.ring == "f64" else torch.int64, device="cuda")
        self.out_n = torch.zeros(self.count, dtype=torch.int64, device="cuda")
        self.offsets = np.concatenate([[0], np.cumsum([max(b, 1) for b in self.bounds])]).astype(np.int64)
        hs = []
        ek, ec = self.out_k.element_size(), self.out_c.element_size()
        for q in range(self.count):
            o = int(self.offsets[q])
            hs.append(pm_poly(self.bounds[q], self.out_n.data_ptr() + 8 * q, self.out_k.data_ptr() + ek * o,
                              self.out_c.data_ptr() + ec * o))
        self.h = (pm_poly * self.count)(*hs)
        self.ws = (workspace or Workspace()).get(self.ws_bytes)

        self.graph = None

    def run(self):
        """One pm_mul_batch call (validation round trip + launches)."""
        _check(lib().pm_mul_batch(ctypes.byref(self.L), self.count, self.cf, self.cg, self.h,
                                  ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream_ptr(self.stream)),
               "pm_mul_batch")

    def prepare_graph(self):
        """Validate once and capture the batch's whole pipeline in a HIP graph."""
        b = ctypes.c_void_p(None)
        _check(lib().pm_batch_prepare(ctypes.byref(self.L), self.count, self.cf, self.cg, self.h,
                                      ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                      _stream_ptr(self.stream), ctypes.byref(b)), "pm_batch_prepare")
        self.graph = b

    def launch_graph(self):
        _check(lib().pm_batch_launch(self.graph, _stream_ptr(self.stream)), "pm_batch_launch")

    def __del__(self):
        g = getattr(self, "graph", None)
        if g is not None and _lib is not None:
            _lib.pm_batch_destroy(g)
            self.graph = None

    def results(self):
        """List of (keys u64, coefs) numpy arrays, after the stream completes."""
        ns = self.out_n.cpu().numpy()
        k = self.out_k.cpu().numpy().view(np.uint64)
        c = self.out_c.cpu().numpy()
        if self.ring == "modp":
            c = c.view(np.uint64)
        out = []
        for q in range(self.count):
            o = int(self.offsets[q])
            out.append((k[o:o + ns[q]], c[o:o + ns[q]]))
        return out


DRAIN_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p,
                            ctypes.c_int64)


def mul_batch_drain(layout, fs, gs, on_result, device_bytes: int, host_bytes: int, stream=None):
    """Products in waves with results drained to pinned host memory while the
    next wave runs; on_result(k, keys, coefs) gets numpy views (valid only
    during the call) of product k's result.  Returns the number of waves."""
    import torch
    L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
    ring = {v: k for k, v in RING_CODE.items()}[L.ring]
    cdt = np.float64 if ring == "f64" else (np.int64 if ring == "i64" else np.uint64)
    count = len(fs)
    cf = (pm_cpoly * max(count, 1))(*[_cpoly(p) for p in fs])
    cg = (pm_cpoly * max(count, 1))(*[_cpoly(p) for p in gs])
    dev = torch.empty(int(device_bytes), dtype=torch.uint8, device="cuda")
    host = torch.empty(int(host_bytes), dtype=torch.uint8, pin_memory=True)
    errors = []

    def cb(_user, k, keys, coefs, n):
        try:
            kk = np.ctypeslib.as_array(keys, shape=(n,)) if n else np.zeros(0, np.uint64)
            cc = (np.ctypeslib.as_array(ctypes.cast(coefs, ctypes.POINTER(ctypes.c_uint64)), shape=(n,)).view(cdt)
                  if n else np.zeros(0, cdt))
            on_result(int(k), kk, cc)
        except Exception as exc:  # raised after the call returns
            errors.append(exc)

    fn = DRAIN_FN(cb)
    waves = ctypes.c_int64(0)
    _check(lib().pm_mul_batch_drain(ctypes.byref(L), count, cf, cg, ctypes.c_void_p(dev.data_ptr()), dev.numel(),
                                    ctypes.c_void_p(host.data_ptr()), host.numel(), fn, None, _stream_ptr(stream),
                                    ctypes.byref(waves)), "pm_mul_batch_drain")
    if errors:
        raise errors[0]
    return int(waves.value)


def mul_batch(layout, fs, gs, workspace=None, stream=None):
    import torch
    call = BatchCall(layout, fs, gs, workspace, stream)
    call.run()
    (stream or torch.cuda.current_stream()).synchronize()
    return call.results()


def last_call_status(stream=None):
    """PM_OK unless the last call on this thread tripped a device-side check."""
    return int(lib().pm_last_call_status(_stream_ptr(stream)))


def last_call_info(stream=None):
    """dict(staged, passes, key_bytes, payload_bytes, box_cells) of the last call."""
    sp, bc = ctypes.c_int64(0), ctypes.c_int64(0)
    ps, kb, vb = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().pm_last_call_info(_stream_ptr(stream), ctypes.byref(sp), ctypes.byref(ps), ctypes.byref(kb),
                                   ctypes.byref(vb), ctypes.byref(bc)), "pm_last_call_info")
    return {"staged": int(sp.value), "passes": int(ps.value), "key_bytes": int(kb.value),
            "payload_bytes": int(vb.value), "box_cells": int(bc.value)}


def profile_enable(on: bool):
    lib().pm_profile_enable(1 if on else 0)


def profile_read():
    """{kernel name: (total ms, launches)} of the recorded launches."""
    out = {}
    n = lib().pm_profile_read(-1, None, 0, None, None)
    for i in range(n):
        buf = ctypes.create_string_buffer(64)
        ms, cnt = ctypes.c_double(0), ctypes.c_int64(0)
        lib().pm_profile_read(i, buf, 64, ctypes.byref(ms), ctypes.byref(cnt))
        out[buf.value.decode()] = (float(ms.value), int(cnt.value))
    return out


def set_tuning(tile_cfg: int = -1, combine: int = -1, allow_dense: bool = True):
    """Autotuner knobs (results never depend on them): tile shape index,
    combine (-1 auto, 0 pair-index sort, 1 LDS tile combine, 2 output-key
    intervals, 3 output-key work items), dense path on/off."""
    _check(lib().pm_set_tuning(tile_cfg, int(combine), int(allow_dense)), "pm_set_tuning")


def plan_from_stats(layout, na, nb, stats):
    """Host-only bound / workspace size (no GPU)."""
    L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
    count = len(na)
    na_a = (ctypes.c_int64 * count)(*na)
    nb_a = (ctypes.c_int64 * count)(*nb)
    st = np.ascontiguousarray(stats, dtype=np.uint64)
    mt = (ctypes.c_int64 * max(count, 1))()
    wb = ctypes.c_int64(0)
    rc = lib().pm_plan_from_stats(ctypes.byref(L), count, na_a, nb_a,
                                  st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), mt, ctypes.byref(wb))
    return rc, [int(mt[i]) for i in range(count)], int(wb.value)


def dense_ceiling(ring: str, stream=None) -> float:
    """Term pairs/s of the dense path's inner loop with no HBM traffic."""
    r = ctypes.c_double(0)
    _check(lib().pm_dense_ceiling(RING_CODE[ring], ctypes.byref(r), _stream_ptr(stream)), "pm_dense_ceiling")
    return float(r.value)


def ival_grid(na: int, nb: int, l: int):
    """Grid samples of the interval split (host only): (rows, cols), (l+1)^2 each."""
    ns = (l + 1) * (l + 1)
    rows = np.zeros(max(ns, 1), np.int64)
    cols = np.zeros(max(ns, 1), np.int64)
    p = ctypes.POINTER(ctypes.c_int64)
    _check(lib().pm_ival_grid(int(na), int(nb), int(l), rows.ctypes.data_as(p), cols.ctypes.data_as(p)),
           "pm_ival_grid")
    return rows[:ns], cols[:ns]


def ival_splitters(fkeys, gkeys, l: int):
    """Splitters S_0 < ... < S_{n-1} of the interval split (host only)."""
    fk = np.ascontiguousarray(fkeys, dtype=np.uint64)
    gk = np.ascontiguousarray(gkeys, dtype=np.uint64)
    out = np.zeros((l + 1) * (l + 1) + 2, np.uint64)
    n = ctypes.c_int64(0)
    u = ctypes.POINTER(ctypes.c_uint64)
    _check(lib().pm_ival_splitters(fk.ctypes.data_as(u), len(fk), gk.ctypes.data_as(u), len(gk), int(l),
                                   out.ctypes.data_as(u), ctypes.byref(n)), "pm_ival_splitters")
    return out[:n.value]


def autotune(layout, f: DevPoly, g: DevPoly, workspace: Workspace | None = None, stream=None):
    """Time the candidate settings on this product; returns (tile_cfg, combine, digits)."""
    call = MulCall(layout, f, g, workspace, stream)
    call.ws = (workspace or Workspace()).get(2 * call.ws_bytes)   # room for the combine setting
    t, c, d = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_int32(-1)
    _check(lib().pm_autotune(ctypes.byref(call.L), ctypes.byref(call.cf), ctypes.byref(call.cg),
                             ctypes.byref(call.h), ctypes.c_void_p(call.ws.data_ptr()), call.ws.numel(), call.sp,
                             ctypes.byref(t), ctypes.byref(c), ctypes.byref(d)), "pm_autotune")
    return int(t.value), int(c.value), int(d.value)


def set_radix(digits: int = -1):
    """Radix digit schedule: -1 automatic, 0 8-bit digits, 1 balanced widths."""
    _check(lib().pm_set_radix(int(digits)), "pm_set_radix")


def autotune_reset():
    lib().pm_autotune_reset()


def autotune_save(path: str):
    """Write the autotuner's remembered choices to a text file."""
    _check(lib().pm_autotune_save(str(path).encode()), "pm_autotune_save")


def autotune_load(path: str):
    """Add the choices of a file written by autotune_save."""
    _check(lib().pm_autotune_load(str(path).encode()), "pm_autotune_load")


class Server:
    """Continuous-batching server (pm_server_*): one HBM arena and a scheduler thread."""

    def __init__(self, hbm_budget_bytes: int, nstreams: int = 4):
        self.h = lib().pm_server_create(int(hbm_budget_bytes), int(nstreams))
        if not self.h:
            raise RuntimeError("pm_server_create failed: " + lib().pm_last_error().decode())
        self.keep = {}

    def submit(self, layout, f: DevPoly, g: DevPoly, out) -> int:
        """Queue h = f * g into out = (keys, coefs, n) tensors; returns a ticket."""
        L = layout if isinstance(layout, pm_layout) else make_layout(*layout)
        hk, hc, hn = out
        h = pm_poly(min(hk.numel(), hc.numel()), hn.data_ptr(), hk.data_ptr(), hc.data_ptr())
        t = ctypes.c_uint64(0)
        _check(lib().pm_server_submit(self.h, ctypes.byref(L), ctypes.byref(_cpoly(f)), ctypes.byref(_cpoly(g)),
                                      ctypes.byref(h), ctypes.byref(t)), "pm_server_submit")
        self.keep[int(t.value)] = (f, g, out)
        return int(t.value)

    def poll(self, ticket: int):
        d, s = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().pm_server_poll(self.h, ticket, ctypes.byref(d), ctypes.byref(s)), "pm_server_poll")
        return bool(d.value), int(s.value)

    def wait(self, ticket: int) -> int:
        s = ctypes.c_int32(0)
        _check(lib().pm_server_wait(self.h, ticket, ctypes.byref(s)), "pm_server_wait")
        return int(s.value)

    def latency_us(self, ticket: int) -> float:
        """Submit-to-completion latency of one completed ticket (microseconds)."""
        v = ctypes.c_double(0)
        _check(lib().pm_server_latency(self.h, ticket, ctypes.byref(v)), "pm_server_latency")
        return float(v.value)

    def latencies_us(self):
        n = lib().pm_server_latencies(self.h, None, 0)
        buf = (ctypes.c_double * max(n, 1))()
        n = lib().pm_server_latencies(self.h, buf, n)
        return [float(buf[i]) for i in range(n)]

    def close(self):
        if self.h:
            lib().pm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
