"""Python access to the CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``libtororacle.so`` (built from
``tor_oracle.c`` by ``oracle/build.py``) and shares nothing with the GPU
library.  What it computes is the plain definition of the Torontonian (Eq. 2)
with a fresh factorisation of every subset's matrix (the square-root-free
form of the Cholesky factor of Sec. 2, det = product of the pivots); the C
source documents it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtororacle.so")

F64 = 0
QUAD = 1
LD = 2  # x87 extended precision (64-bit significand)

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # noqa: F401  (only the oracle's own build step)
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_tor.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_long, ctypes.c_int,
                               ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_double)]
    lib.oracle_tor.restype = ctypes.c_int
    lib.oracle_det.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_long, ctypes.c_uint64,
                               ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_det.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


@dataclass
class OracleResult:
    hi: float
    lo: float
    sum_abs: float
    count: int
    sum_sq: float = float("nan")  # sum of t^2

    @property
    def value(self) -> float:
        return self.hi + self.lo

    @property
    def cancellation(self) -> float:
        """R = sum |t| / |Tor|."""
        v = abs(self.hi)
        return float("inf") if v == 0.0 else self.sum_abs / v


def _as_c128(O):
    O = np.ascontiguousarray(np.asarray(O, dtype=np.complex128))
    if O.ndim != 2 or O.shape[0] != O.shape[1] or O.shape[0] % 2:
        raise ValueError("O must be a 2n x 2n matrix")
    return O


def tor(O, mode: int = F64, threads: int = 0, fix_mask: int = 0, fix_val: int = 0) -> OracleResult:
    """Sum of (-1)^(n-|Z|)/sqrt(det (I-O)_Z) over Z with (Z & fix_mask) == fix_val."""
    O = _as_c128(O)
    n = O.shape[0] // 2
    out = (ctypes.c_double * 5)()
    rc = _load().oracle_tor(n, O.ctypes.data if n else None, max(2 * n, 1), mode, threads,
                            fix_mask, fix_val, out)
    if rc != 0:
        raise OracleError({-1: "invalid argument", -2: "I - O not positive definite",
                           -3: "out of memory"}.get(rc, str(rc)))
    return OracleResult(out[0], out[1], out[2], int(out[3]), out[4])


def det(O, Z: int, mode: int = F64):
    """(det (I-O)_Z, signed term) for one subset bitmask Z."""
    O = _as_c128(O)
    n = O.shape[0] // 2
    out = (ctypes.c_double * 2)()
    rc = _load().oracle_det(n, O.ctypes.data if n else None, max(2 * n, 1), Z, mode, out)
    if rc != 0:
        raise OracleError(str(rc))
    return out[0], out[1]
