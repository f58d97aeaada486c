"""Binding of libaop_cpu (include/aop_cpu.h): the FFT nonlinear-stencil method
on host cores with OpenMP tasks, the comparison path in the paper's own
setting.  Argument marshalling only; raises if the library is missing."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from paper_2303_02317_amd.binding import options_array

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaop_cpu.so")
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libaop_cpu.so is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.aop_cpu_price_batch.restype = ctypes.c_int32
        lib.aop_cpu_price_batch.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                            P, P, P, ctypes.c_int64]
        _lib = lib
    return _lib


def price_batch(opts, threads: int = 0, base: int = 0, lam: float = 1.0 / 3.0, boundary: bool = False):
    """(prices, status, boundaries or None) for a list of option dicts."""
    n = len(opts)
    price = np.empty(max(n, 1), dtype=np.float64)
    status = np.zeros(max(n, 1), dtype=np.int32)
    stride = max(int(o["T"]) for o in opts) + 1 if (boundary and n) else 0
    bnd = np.empty((max(n, 1), max(stride, 1)), dtype=np.int64) if boundary else None
    rc = load().aop_cpu_price_batch(options_array(opts), n, int(threads), int(base), float(lam),
                                    price.ctypes.data, status.ctypes.data,
                                    bnd.ctypes.data if bnd is not None else None, stride)
    if rc != 0:
        raise RuntimeError("aop_cpu_price_batch failed with status %d" % rc)
    return price[:n], status[:n], (bnd[:n] if bnd is not None else None)
