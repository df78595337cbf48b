"""The paper's parallel CPU search (Section 3: private deques, receiver-initiated
stealing, task groups, token-ring termination) on the host cores: a
measurement baseline beside the GPU search, never used by it."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _build

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_build.CPU_WS_SO):
            _build.build_cpu_baseline()
        L = ctypes.CDLL(_build.CPU_WS_SO)
        P, U32, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.sge_cpu_count.restype = I32
        L.sge_cpu_count.argtypes = [U32, P, P, P, U32, P, P, P, I32, I32, I32, I32, P, ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a if a.size else np.zeros(1, dtype=np.uint32)


def count(pattern, target, mode: int, labelled: bool, threads: int, group: int = 4) -> dict:
    """Undirected graphs.  Returns {matches, states, steals, seconds}."""
    p = [_u32(pattern.row_ptr), _u32(pattern.col), _u32(pattern.labels)]
    t = [_u32(target.row_ptr), _u32(target.col), _u32(target.labels)]
    cnt = np.zeros(3, dtype=np.uint64)
    sec = ctypes.c_double(0)
    rc = lib().sge_cpu_count(pattern.n, *[a.ctypes.data for a in p], target.n, *[a.ctypes.data for a in t],
                             int(mode), int(bool(labelled)), int(threads), int(group), cnt.ctypes.data,
                             ctypes.byref(sec))
    if rc != 0:
        raise ValueError("sge_cpu_count rejected the input")
    return dict(matches=int(cnt[0]), states=int(cnt[1]), steals=int(cnt[2]), seconds=sec.value)
