"""CPU oracle for the sparse polynomial product -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps `oracle.c` (plain C, single-threaded, built
with gcc) through ctypes and shares nothing with the GPU library.

The computed result is the plain definition of the product (Section 2 of the
paper, problem statement and Fig. 1): every pairwise term product, equal
monomials grouped, like terms summed, zero terms dropped, output sorted
ascending by packed monomial key.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, EUNSORTED, EOVERFLOW, ERANGE, ECAPACITY, ENOMEM, EINT64 = 0, -1, -2, -3, -4, -5, -6, -9
RING_CODE = {"modp": 0, "f64": 1, "i64": 2, "modq": 3, "z192": 4}
COEF_DTYPE = {"modp": np.uint64, "f64": np.float64, "i64": np.int64, "modq": np.uint64, "z192": np.uint64}
COEF_WORDS = {"z192": 3}    # coefficient words per term (1 for the other rings)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_mul.restype = ctypes.c_int
        L.oracle_mul.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, i64p]
        L.oracle_validate.restype = ctypes.c_int
        L.oracle_validate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_bound.restype = ctypes.c_int
        L.oracle_bound.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_void_p, i64p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, (a.ctypes.data if a.size else None)


def validate(nvars, bits, ring, fk, fc, gk, gc) -> int:
    fk, pfk = _arr(fk, np.uint64)
    gk, pgk = _arr(gk, np.uint64)
    fc, pfc = _arr(fc, COEF_DTYPE[ring])
    gc, pgc = _arr(gc, COEF_DTYPE[ring])
    return lib().oracle_validate(nvars, bits, RING_CODE[ring], fk.size, pfk, pfc, gk.size, pgk, pgc)


def mul_arrays(nvars, bits, ring, fk, fc, gk, gc, cap=None):
    """Returns (keys u64, coefs, abssum or None).  Raises OracleError."""
    fk, pfk = _arr(fk, np.uint64)
    gk, pgk = _arr(gk, np.uint64)
    fc, pfc = _arr(fc, COEF_DTYPE[ring])
    gc, pgc = _arr(gc, COEF_DTYPE[ring])
    L = lib()
    nh = ctypes.c_int64(0)
    if cap is None:
        b = ctypes.c_int64(0)
        rc = L.oracle_bound(nvars, bits, fk.size, pfk, gk.size, pgk, ctypes.byref(b))
        if rc != OK:
            raise OracleError(rc)
        cap = int(b.value)
    hk = np.zeros(max(cap, 1), dtype=np.uint64)
    w = COEF_WORDS.get(ring, 1)
    hc = np.zeros((max(cap, 1), w) if w > 1 else max(cap, 1), dtype=COEF_DTYPE[ring])
    ha = np.zeros(max(cap, 1), dtype=np.float64) if ring == "f64" else None
    rc = L.oracle_mul(nvars, bits, RING_CODE[ring], fk.size, pfk, pfc, gk.size, pgk, pgc,
                      cap, hk.ctypes.data, hc.ctypes.data, ha.ctypes.data if ha is not None else None,
                      ctypes.byref(nh))
    if rc != OK:
        raise OracleError(rc)
    n = int(nh.value)
    return hk[:n].copy(), hc[:n].copy(), (ha[:n].copy() if ha is not None else None)


def mul(f, g):
    """Product of two workload polynomials (objects with .layout, .keys, .coefs)."""
    lay = f.layout
    return mul_arrays(lay.nvars, lay.bits, lay.ring, f.keys, f.coefs, g.keys, g.coefs)
