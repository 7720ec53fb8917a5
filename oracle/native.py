"""Build and call the C parts of the oracle (TEST INFRASTRUCTURE ONLY).

ryser_c.c (plain Ryser) and hper_c.c (Algorithm H_per with Ryser leaves) are compiled
with gcc into oracle/_build/liboracle_c.so. Both compute exact permanents of dense
non-negative integer matrices in 128-bit wrap-around arithmetic (exact below 2^128).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(_HERE, "ryser_c.c"), os.path.join(_HERE, "hper_c.c")]
LIB = os.path.join(_HERE, "_build", "liboracle_c.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle sources with gcc (always when ``force``, else only if stale)."""
    stale = not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SRCS)
    if force or stale:
        os.makedirs(os.path.dirname(LIB), exist_ok=True)
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", *SRCS, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        for name in ("oracle_ryser_batch", "oracle_hper_batch"):
            fn = getattr(_lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_int]
    return _lib


def _call(name, mats, threads, dtype, max_order):
    lib = _load()
    mats = [np.ascontiguousarray(np.asarray(m, dtype=dtype)) for m in mats]
    for m in mats:
        if m.ndim != 2 or m.shape[0] != m.shape[1] or m.shape[0] > max_order:
            raise ValueError("square matrices of order <= %d expected" % max_order)
    order = np.array([m.shape[0] for m in mats], dtype=np.int32)
    sizes = np.array([m.size for m in mats], dtype=np.int64)
    offset = (np.concatenate([[0], np.cumsum(sizes)[:-1]]) if mats else np.zeros(0)).astype(np.int64)
    entries = np.concatenate([m.ravel() for m in mats] + [np.zeros(1, dtype)])
    lo = np.zeros(max(len(mats), 1), dtype=np.uint64)
    hi = np.zeros(max(len(mats), 1), dtype=np.uint64)
    rc = getattr(lib, name)(len(mats), order.ctypes.data, offset.ctypes.data, entries.ctypes.data,
                            lo.ctypes.data, hi.ctypes.data, int(threads))
    if rc == -2:
        raise OverflowError("an expanded entry exceeded 2^62")
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments")
    return [int(h) << 64 | int(l) for l, h in zip(lo.tolist()[:len(mats)], hi.tolist()[:len(mats)])]


def ryser_batch(mats, threads: int = 1) -> list[int]:
    """per(A) by plain Ryser for each dense matrix (order <= 40), on ``threads`` threads."""
    return _call("oracle_ryser_batch", mats, threads, np.uint32, 40)


def hper_batch(mats, threads: int = 1) -> list[int]:
    """per(A) by Algorithm H_per (expansion (2) + Ryser leaves) for each matrix (order <= 128)."""
    return _call("oracle_hper_batch", mats, threads, np.uint64, 128)
