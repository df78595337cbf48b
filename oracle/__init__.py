"""Python access to the oracle (plain single-threaded CPU reference).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library's product path.  The C
source is compiled with gcc into ``oracle/_build/liboracle.so``.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sge_oracle.c")
SO = os.path.join(HERE, "_build", "liboracle.so")

RI, RIDS, RIDS_SI, RIDS_SI_FC = 0, 1, 2, 3
OK, ABORTED = 0, 2

_lib = None


def build() -> str:
    os.makedirs(os.path.dirname(SO), exist_ok=True)
    tmp = SO + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp], check=True)
    os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = ctypes.CDLL(SO)
        p = ctypes.c_void_p
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_uint32, p, p, p, ctypes.c_uint32, p, p, p, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, p, ctypes.c_uint64, p]
        L.oracle_plan.restype = ctypes.c_int
        L.oracle_plan.argtypes = [ctypes.c_uint32, p, p, p, ctypes.c_uint32, p, p, p, ctypes.c_int, ctypes.c_int,
                                  p, p, p, p]
        L.oracle_run_ex.restype = ctypes.c_int
        L.oracle_run_ex.argtypes = [ctypes.c_uint32, p, p, p, p, ctypes.c_int, ctypes.c_uint32, p, p, p, p,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, p, ctypes.c_uint64, p]
        L.oracle_plan_ex.restype = ctypes.c_int
        L.oracle_plan_ex.argtypes = [ctypes.c_uint32, p, p, p, p, ctypes.c_int, ctypes.c_uint32, p, p, p, p,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, p, p, p, p]
        L.oracle_forward_check.restype = ctypes.c_int
        L.oracle_forward_check.argtypes = [ctypes.c_uint32, ctypes.c_uint32, p]
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a if a.size else np.zeros(1, dtype=np.uint32)


def _graph_args(g):
    """CSR, node labels, edge labels (or NULL) and the directed flag of a graph."""
    rp, col = _u32(g.row_ptr), _u32(g.col)
    lab = _u32(g.labels if g.labels is not None else np.zeros(g.n, dtype=np.uint32))
    el = getattr(g, "elabels", None)
    el = None if el is None else _u32(el)
    directed = int(bool(getattr(g, "directed", False)))
    return (rp, col, lab, el), [rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                None if el is None else el.ctypes.data, directed]


def run(pattern, target, mode: int, labelled: bool, state_cap: int = 0, rows: bool = False,
        cap_rows: int = 1 << 20, root_range=(0, 0xFFFFFFFF)) -> dict:
    """Enumerate; returns {status, matches, states, candidates, alg_bytes,
    dense_bytes, rows?}.  The byte counts are those of a count-only search (an
    enumeration also writes 4k bytes per match).  root_range restricts the
    first node of the order to target nodes in [lo, hi)."""
    keep_p, pa = _graph_args(pattern)
    keep_t, ta = _graph_args(target)
    cnt = np.zeros(5, dtype=np.uint64)
    buf = np.zeros((cap_rows if rows else 0, max(pattern.n, 1)), dtype=np.uint32)
    rc = lib().oracle_run_ex(pattern.n, *pa, target.n, *ta, int(mode), int(bool(labelled)), int(state_cap),
                             int(root_range[0]), int(root_range[1]),
                             buf.ctypes.data if rows else None, cap_rows if rows else 0, cnt.ctypes.data)
    if rc < 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    out = dict(status=rc, matches=int(cnt[0]), states=int(cnt[1]), candidates=int(cnt[2]),
               alg_bytes=int(cnt[3]), dense_bytes=int(cnt[4]))
    if rows:
        nr = min(out["matches"], cap_rows)
        out["rows"] = buf[:nr, :pattern.n].copy()
    return out


def plan(pattern, target, mode: int, labelled: bool) -> dict:
    """Ordering, parents and final domains (bool array [k, n], or None in RI)."""
    keep_p, pa = _graph_args(pattern)
    keep_t, ta = _graph_args(target)
    k, n = pattern.n, target.n
    order = np.zeros(max(k, 1), dtype=np.uint32)
    parent = np.zeros(max(k, 1), dtype=np.int32)
    dom = np.zeros((max(k, 1), max(n, 1)), dtype=np.uint8)
    empty = ctypes.c_int(0)
    rc = lib().oracle_plan_ex(k, *pa, n, *ta, int(mode), int(bool(labelled)), order.ctypes.data,
                              parent.ctypes.data, dom.ctypes.data if mode != RI else None, ctypes.byref(empty))
    if rc < 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return dict(order=order[:k].copy(), parent=parent[:k].copy(), empty=bool(empty.value),
                domains=(dom[:k, :n].astype(bool) if mode != RI else None))


def forward_check(domains: np.ndarray) -> tuple[bool, np.ndarray]:
    """Forward checking on a bool [k, n] domain array; returns (emptied, result)."""
    d = np.ascontiguousarray(domains.astype(np.uint8))
    k, n = d.shape
    rc = lib().oracle_forward_check(k, n, d.ctypes.data)
    if rc < 0:
        raise ValueError("k > 64")
    return bool(rc), d.astype(bool)


def rows_digest(rows: np.ndarray, k: int) -> str:
    """SHA-256 of the lexicographically sorted rows, each k little-endian uint32."""
    r = np.asarray(rows, dtype=np.uint32).reshape(-1, k) if k else np.zeros((0, 0), dtype=np.uint32)
    if r.shape[0] > 1 and k:
        r = r[np.lexsort(r.T[::-1])]
    return hashlib.sha256(np.ascontiguousarray(r).astype("<u4").tobytes()).hexdigest()
