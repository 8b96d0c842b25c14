"""ctypes wrapper around the serial scan form in ``oracle/scan.c``.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

``Prepared`` holds the one-time integer/KM preparation computed by the
oracle's own code (``oracle.prep``, ``oracle.km``); ``coordinate`` evaluates
g', g'' and l for one coordinate in O(N) with compensated sums (Sec. 2.7).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import km, prep

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan.c")
_LIB = os.path.join(_HERE, "_scan.so")
_lib = None


def build(force=True):
    """Compile ``scan.c`` with gcc (no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_cox_scan.argtypes = [ctypes.c_int64, dp, ip, dp, dp, dp]
        lib.oracle_cox_scan.restype = ctypes.c_int
        lib.oracle_fg_scan.argtypes = [ctypes.c_int64, dp, ip, dp, dp, dp, dp]
        lib.oracle_fg_scan.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class Prepared:
    """Sorted view of one data set (Sec. 2.7 ordering; Sec. 2.2 KM)."""

    def __init__(self, model, y, status):
        self.model = model
        y = np.asarray(y, dtype=np.float64)
        status = np.asarray(status).astype(np.int64)
        self.n = y.size
        self.order = prep.order(y)
        self.inv = np.empty_like(self.order)
        self.inv[self.order] = np.arange(self.n)
        self.y = np.ascontiguousarray(y[self.order])
        self.status = np.ascontiguousarray(status[self.order])
        self.ev = prep.event_indicator(model, self.status)
        if model == "fg":
            t, v = km.km_censoring(y, status)
            self.gy = np.ascontiguousarray(km.km_eval(t, v, self.y))
        else:
            self.gy = None

    def coordinate_sorted(self, eta_s, x_s):
        """g', g'', l from arrays already in sorted order."""
        lib = _load()
        eta_s = np.ascontiguousarray(eta_s, dtype=np.float64)
        x_s = np.ascontiguousarray(x_s, dtype=np.float64)
        out = np.zeros(10, dtype=np.float64)
        if self.model == "cox":
            rc = lib.oracle_cox_scan(self.n, _dp(self.y), _ip(self.ev),
                                     _dp(eta_s), _dp(x_s), _dp(out))
        else:
            rc = lib.oracle_fg_scan(self.n, _dp(self.y), _ip(self.status),
                                    _dp(eta_s), _dp(x_s), _dp(self.gy),
                                    _dp(out))
        if rc != 0:
            raise MemoryError("oracle scan failed")
        return {"g1": out[0], "g2": out[1], "loglik": out[2],
                "A": out[3], "B": out[4], "L": out[5],
                "scale_g1": out[9] + out[6], "scale_g2": out[7],
                "scale_L": out[8]}

    def coordinate(self, eta, xj):
        """g', g'', l from arrays in the original subject order."""
        eta = np.asarray(eta, dtype=np.float64)
        xj = np.asarray(xj, dtype=np.float64)
        return self.coordinate_sorted(eta[self.order], xj[self.order])


def scan(model, y, status, eta, xj):
    """One-shot helper: prepare and evaluate one coordinate."""
    return Prepared(model, y, status).coordinate(eta, xj)
