"""ctypes binding of the oracle's C direct sums (greens.c), plus its build.

Test infrastructure only: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the library.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "greens.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force=False):
    """Compile greens.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            L.oracle_history.argtypes = [i64, dp, dp, i64, dp, dp, dp, i64, dp, dp, dp, dp, dp, dp,
                                         ctypes.c_double, dp, dp, dp]
            L.oracle_history.restype = None
            L.oracle_gh_vec.argtypes = [i64, dp, ctypes.c_double, dp]
            L.oracle_ein_vec.argtypes = [i64, dp, dp]
            L.oracle_kd.argtypes = [ctypes.c_double] * 5
            L.oracle_kd.restype = ctypes.c_double
            L.oracle_num_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def ein(z):
    z = _c(np.atleast_1d(z))
    out = np.empty_like(z)
    lib().oracle_ein_vec(z.size, _p(z), _p(out))
    return out


def gh(d2, delta):
    d2 = _c(np.atleast_1d(d2))
    out = np.empty_like(d2)
    lib().oracle_gh_vec(d2.size, _p(d2), float(delta), _p(out))
    return out


def kd(dx, dy, nx, ny, delta):
    return lib().oracle_kd(float(dx), float(dy), float(nx), float(ny), float(delta))


def num_threads():
    return lib().oracle_num_threads()


def history(tx, ty, sx=None, sy=None, c=None, bx=None, by=None, bnx=None, bny=None,
            s=None, m=None, delta=None):
    """Direct sums: returns (V_H, S_H, D_H) arrays (None where the density is None)."""
    tx, ty = _c(tx), _c(ty)
    n = tx.size
    sx, sy, c = _c(sx), _c(sy), _c(c)
    bx, by, bnx, bny, s, m = _c(bx), _c(by), _c(bnx), _c(bny), _c(s), _c(m)
    oV = np.zeros(n) if c is not None else None
    oS = np.zeros(n) if s is not None else None
    oD = np.zeros(n) if m is not None else None
    ns = 0 if c is None else c.size
    nb = 0 if (s is None and m is None) else bx.size
    lib().oracle_history(n, _p(tx), _p(ty), ns, _p(sx), _p(sy), _p(c), nb, _p(bx), _p(by),
                         _p(bnx), _p(bny), _p(s), _p(m), float(delta), _p(oV), _p(oS), _p(oD))
    return oV, oS, oD
