"""Thin ctypes binding of the C ABI in ``include/sge.h`` (argument marshalling only).

Every step of the search runs in the native library ``_lib/libsge.so``: input
validation in C++ when graphs are loaded, the plan and the search in HIP
kernels for gfx950.  If the library is
missing it is built in-tree; if it cannot be loaded an error is raised -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsge.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_OVERFLOW, E_ABORTED, E_BUSY, E_HANDLE = 0, -1, -2, -3, -4, -5, -6, -7
RI, RIDS, RIDS_SI, RIDS_SI_FC = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_OVERFLOW", -5: "E_ABORTED",
                -6: "E_BUSY", -7: "E_HANDLE"}

EXPORTS = [
    "sge_create", "sge_destroy", "sge_last_error", "sge_load_target", "sge_unload_target", "sge_load_pattern",
    "sge_unload_pattern", "sge_load_target_ex", "sge_load_pattern_ex", "sge_plan_host_ex", "sge_set_labelled", "sge_set_mode", "sge_set_state_cap", "sge_set_root_range",
    "sge_count", "sge_enumerate", "sge_batch_run", "sge_set_batch_policy", "sge_serve_start", "sge_serve_submit",
    "sge_serve_poll", "sge_serve_stop", "sge_plan_host", "sge_plan_device", "sge_set_plan_location", "sge_set_tuning",
    "sge_set_time_limit", "sge_last_launch_timing", "sge_last_launch_occupancy", "sge_set_blocks_per_cu",
    "sge_last_kernel_ms", "sge_set_count_bytes", "sge_set_checks", "sge_count_noalloc",
]


class c_result(ctypes.Structure):
    _fields_ = [("matches", ctypes.c_uint64), ("states", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_uint64), ("steals", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("ms_prep", ctypes.c_double), ("ms_search", ctypes.c_double)]


class c_job(ctypes.Structure):
    _fields_ = [("target", ctypes.c_uint32), ("pattern", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("labelled", ctypes.c_int32)]


@dataclasses.dataclass
class Result:
    status: int
    matches: int
    states: int
    candidates: int
    alg_bytes: int
    steals: int
    steps: int
    ms_prep: float
    ms_search: float

    @staticmethod
    def of(st: int, r: c_result) -> "Result":
        return Result(st, r.matches, r.states, r.candidates, r.alg_bytes, r.steals, r.steps, r.ms_prep,
                      r.ms_search)


# numpy layouts of sge_job and sge_result, for batches marshalled without
# per-job Python objects
JOB_DTYPE = np.dtype([("target", "<u4"), ("pattern", "<u4"), ("mode", "<i4"), ("labelled", "<i4")])
RESULT_DTYPE = np.dtype([("matches", "<u8"), ("states", "<u8"), ("candidates", "<u8"), ("alg_bytes", "<u8"),
                         ("steals", "<u8"), ("steps", "<u8"), ("ms_prep", "<f8"), ("ms_search", "<f8")])
assert JOB_DTYPE.itemsize == ctypes.sizeof(c_job) and RESULT_DTYPE.itemsize == ctypes.sizeof(c_result)


def job_array(jobs) -> np.ndarray:
    """(target, pattern, mode, labelled) tuples -> a contiguous sge_job array (reusable across runs)."""
    if isinstance(jobs, np.ndarray) and jobs.dtype == JOB_DTYPE:
        return np.ascontiguousarray(jobs)
    return np.array([(int(t), int(p), int(m), int(bool(l))) for t, p, m, l in jobs], dtype=JOB_DTYPE)


class BatchResults:
    """Per-job counters of one batch: columns as numpy arrays (``.states``,
    ``.matches``, ...), or one Result per job by index or iteration."""

    def __init__(self, status: int, array: np.ndarray):
        self.status = status
        self.array = array

    def __len__(self) -> int:
        return len(self.array)

    def __getitem__(self, i: int) -> "Result":
        r = self.array[i]
        return Result(self.status, int(r["matches"]), int(r["states"]), int(r["candidates"]), int(r["alg_bytes"]),
                      int(r["steals"]), int(r["steps"]), float(r["ms_prep"]), float(r["ms_search"]))

    def __iter__(self):
        return (self[i] for i in range(len(self)))

    def __getattr__(self, name):
        if name in RESULT_DTYPE.names:
            return self.array[name]
        raise AttributeError(name)


class SgeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import _build
            _build.build_sge()
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "sge_create": (I32, [I32, P, ctypes.POINTER(P)]),
            "sge_destroy": (None, [P]),
            "sge_last_error": (ctypes.c_char_p, [P]),
            "sge_load_target": (I32, [P, U32, P, P, P, ctypes.POINTER(U32)]),
            "sge_unload_target": (I32, [P, U32]),
            "sge_load_pattern": (I32, [P, U32, P, P, P, ctypes.POINTER(U32)]),
            "sge_load_target_ex": (I32, [P, U32, P, P, P, P, I32, ctypes.POINTER(U32)]),
            "sge_load_pattern_ex": (I32, [P, U32, P, P, P, P, I32, ctypes.POINTER(U32)]),
            "sge_plan_host_ex": (I32, [U32, P, P, P, P, I32, U32, P, P, P, P, I32, I32, I32, P, P, P,
                                       ctypes.POINTER(I32)]),
            "sge_unload_pattern": (I32, [P, U32]),
            "sge_set_labelled": (I32, [P, I32]),
            "sge_set_mode": (I32, [P, I32]),
            "sge_set_state_cap": (I32, [P, U64]),
            "sge_set_root_range": (I32, [P, U32, U32]),
            "sge_count": (I32, [P, U32, U32, ctypes.POINTER(c_result)]),
            "sge_enumerate": (I32, [P, U32, U32, P, U64, ctypes.POINTER(c_result)]),
            "sge_batch_run": (I32, [P, U32, P, P]),
            "sge_set_batch_policy": (I32, [P, I32]),
            "sge_serve_start": (I32, [P, U32, U64]),
            "sge_serve_submit": (I32, [P, ctypes.POINTER(c_job), ctypes.POINTER(U64)]),
            "sge_serve_poll": (I32, [P, U64, ctypes.POINTER(c_result)]),
            "sge_serve_stop": (I32, [P]),
            "sge_plan_host": (I32, [U32, P, P, P, U32, P, P, P, I32, I32, P, P, P, ctypes.POINTER(I32)]),
            "sge_plan_device": (I32, [P, U32, U32, I32, I32, P, P, P, ctypes.POINTER(U32), ctypes.POINTER(I32)]),
            "sge_set_tuning": (I32, [P, I32, U32, I32, I32]),
            "sge_set_plan_location": (I32, [P, I32]),
            "sge_set_time_limit": (I32, [P, U64]),
            "sge_last_launch_timing": (I32, [P, P]),
            "sge_last_launch_occupancy": (I32, [P, P, P]),
            "sge_set_blocks_per_cu": (I32, [P, I32]),
            "sge_last_kernel_ms": (I32, [P, ctypes.POINTER(ctypes.c_double)]),
            "sge_set_count_bytes": (I32, [P, I32]),
            "sge_set_checks": (I32, [P, I32]),
            "sge_count_noalloc": (I32, [P, U32, U32, ctypes.POINTER(c_result)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a if a.size else np.zeros(1, dtype=np.uint32)


def _elabels(g):
    el = getattr(g, "elabels", None)
    return None if el is None else _u32(el)


def plan_host(pattern, target, mode: int, labelled: bool) -> dict:
    """The library's host plan (order, parents, domains as bool [k, n]); no device use."""
    k, n = pattern.n, target.n
    prp, pcol, plab = _u32(pattern.row_ptr), _u32(pattern.col), _u32(pattern.labels)
    trp, tcol, tlab = _u32(target.row_ptr), _u32(target.col), _u32(target.labels)
    pel, tel = _elabels(pattern), _elabels(target)
    W = (n + 63) // 64
    order = np.zeros(max(k, 1), np.uint32)
    parent = np.zeros(max(k, 1), np.int32)
    dom = np.zeros(max(k * W, 1), np.uint64)
    empty = ctypes.c_int(0)
    st = lib().sge_plan_host_ex(k, prp.ctypes.data, pcol.ctypes.data, plab.ctypes.data,
                                None if pel is None else pel.ctypes.data, int(getattr(pattern, "directed", False)),
                                n, trp.ctypes.data, tcol.ctypes.data, tlab.ctypes.data,
                                None if tel is None else tel.ctypes.data, int(getattr(target, "directed", False)),
                                mode, int(labelled), order.ctypes.data, parent.ctypes.data, dom.ctypes.data,
                                ctypes.byref(empty))
    if st != OK:
        raise SgeError(st, "sge_plan_host rejected the input")
    domains = None
    if mode != RI and k:
        bits = np.unpackbits(dom[:k * W].view(np.uint8).reshape(k, W * 8), axis=1, bitorder="little")
        domains = bits[:, :n].astype(bool)
    return dict(order=order[:k].copy(), parent=parent[:k].copy(), empty=bool(empty.value), domains=domains)


class Context:
    """One library context on one HIP device, ordered on one stream."""

    def __init__(self, device: int = 0, stream=None):
        self._L = lib()
        h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        st = self._L.sge_create(device, s, ctypes.byref(h))
        if st != OK:
            raise SgeError(st, "sge_create failed (no usable HIP device?)")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._L.sge_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int, what: str) -> int:
        if st != OK:
            msg = self._L.sge_last_error(self._h)
            raise SgeError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def last_launch_timing(self):
        """(kernel ms, ms until the last task finished, ms until termination was detected)."""
        out = (ctypes.c_double * 3)()
        self._check(self._L.sge_last_launch_timing(self._h, ctypes.addressof(out)), "sge_last_launch_timing")
        return tuple(out)

    def last_kernel_ms(self) -> float:
        """HIP-event time (ms) of the last launch's search kernel."""
        ms = ctypes.c_double()
        self._check(self._L.sge_last_kernel_ms(self._h, ctypes.byref(ms)), "sge_last_kernel_ms")
        return ms.value

    def set_count_bytes(self, on: bool):
        """Count each search's algorithmic bytes (Result.alg_bytes); on by default."""
        self._check(self._L.sge_set_count_bytes(self._h, int(bool(on))), "sge_set_count_bytes")

    def set_checks(self, on: bool):
        """Verify, every search step, that a unit's lanes agree on its state (for testing)."""
        self._check(self._L.sge_set_checks(self._h, int(bool(on))), "sge_set_checks")

    def last_launch_occupancy(self):
        """(sum over units of the ms each held a task, units that entered the
        search loop) for the last launch."""
        busy = ctypes.c_double()
        units = ctypes.c_uint32()
        self._check(self._L.sge_last_launch_occupancy(self._h, ctypes.byref(busy), ctypes.byref(units)),
                    "sge_last_launch_occupancy")
        return busy.value, units.value

    def plan_device(self, target: int, pattern: int, k: int, n: int, mode: int, labelled: bool) -> dict:
        """The plan the device computes before a search: order, parents, the
        number of root candidates and (RI-DS modes) domains as bool [k, n]."""
        W = (n + 63) // 64
        order = np.zeros(max(k, 1), np.uint32)
        parent = np.zeros(max(k, 1), np.int32)
        dom = np.zeros(max(k * W, 1), np.uint64)
        nroot = ctypes.c_uint32(0)
        empty = ctypes.c_int(0)
        self._check(self._L.sge_plan_device(self._h, target, pattern, mode, int(bool(labelled)), order.ctypes.data,
                                            parent.ctypes.data, dom.ctypes.data, ctypes.byref(nroot),
                                            ctypes.byref(empty)), "sge_plan_device")
        domains = None
        if mode != RI and k and not empty.value:
            bits = np.unpackbits(dom[:k * W].view(np.uint8).reshape(k, W * 8), axis=1, bitorder="little")
            domains = bits[:, :n].astype(bool)
        return dict(order=order[:k].copy(), parent=parent[:k].copy(), nroot=int(nroot.value),
                    empty=bool(empty.value), domains=domains)

    def last_error(self) -> str:
        m = self._L.sge_last_error(self._h)
        return m.decode() if m else ""

    def _load(self, fn, g, what):
        """Graphs with edge labels (``elabels``) or ``directed`` set go through the _ex loaders."""
        rp, col = _u32(g.row_ptr), _u32(g.col)
        lab = None if g.labels is None else _u32(g.labels)
        el = _elabels(g)
        out = ctypes.c_uint32()
        self._check(fn(self._h, g.n, rp.ctypes.data, col.ctypes.data, None if lab is None else lab.ctypes.data,
                       None if el is None else el.ctypes.data, int(bool(getattr(g, "directed", False))),
                       ctypes.byref(out)), what)
        return out.value

    def load_target(self, g) -> int:
        return self._load(self._L.sge_load_target_ex, g, "sge_load_target")

    def load_pattern(self, g) -> int:
        return self._load(self._L.sge_load_pattern_ex, g, "sge_load_pattern")

    def unload_target(self, h: int):
        self._check(self._L.sge_unload_target(self._h, h), "sge_unload_target")

    def unload_pattern(self, h: int):
        self._check(self._L.sge_unload_pattern(self._h, h), "sge_unload_pattern")

    def set_labelled(self, labelled: bool):
        self._check(self._L.sge_set_labelled(self._h, int(bool(labelled))), "sge_set_labelled")

    def set_mode(self, mode: int):
        self._check(self._L.sge_set_mode(self._h, int(mode)), "sge_set_mode")

    def set_state_cap(self, cap: int):
        self._check(self._L.sge_set_state_cap(self._h, int(cap)), "sge_set_state_cap")

    def set_time_limit(self, ms: int):
        self._check(self._L.sge_set_time_limit(self._h, int(ms)), "sge_set_time_limit")

    def set_root_range(self, lo: int = 0, hi: int = 0xFFFFFFFF):
        self._check(self._L.sge_set_root_range(self._h, int(lo), int(hi)), "sge_set_root_range")

    def set_tuning(self, lanes: int = 0, root_chunk: int = 0, donate: int = 1, dense: int = -1):
        """donate: 0 off, 1 default period, N > 1 at most one donation per N steps of a unit."""
        self._check(self._L.sge_set_tuning(self._h, lanes, root_chunk, int(donate), dense), "sge_set_tuning")

    def set_blocks_per_cu(self, blocks_per_cu: int):
        """Resident search blocks per CU: 0 automatic, N >= 1 at most N."""
        self._check(self._L.sge_set_blocks_per_cu(self._h, int(blocks_per_cu)), "sge_set_blocks_per_cu")

    def set_plan_location(self, where: int):
        """-1 automatic, 0 host, 1 device."""
        self._check(self._L.sge_set_plan_location(self._h, where), "sge_set_plan_location")

    def set_batch_policy(self, policy: int):
        self._check(self._L.sge_set_batch_policy(self._h, policy), "sge_set_batch_policy")

    def count(self, target: int, pattern: int, allow=(OK,)) -> Result:
        r = c_result()
        st = self._L.sge_count(self._h, target, pattern, ctypes.byref(r))
        if st not in allow:
            self._check(st, "sge_count")
        return Result.of(st, r)

    def count_noalloc(self, target: int, pattern: int, allow=(OK,)) -> Result:
        """sge_count with every device buffer in the library's static scratch array."""
        r = c_result()
        st = self._L.sge_count_noalloc(self._h, target, pattern, ctypes.byref(r))
        if st not in allow:
            self._check(st, "sge_count_noalloc")
        return Result.of(st, r)

    def enumerate(self, target: int, pattern: int, k: int, cap_rows: int = 1 << 20, rows=None, allow=(OK,)):
        """Returns (Result, rows).  `rows` may be a device tensor (torch, uint32-compatible int32,
        shape [cap_rows, k]); by default a host numpy array is used."""
        r = c_result()
        if rows is None:
            buf = np.zeros((max(cap_rows, 1), max(k, 1)), dtype=np.uint32)
            ptr = buf.ctypes.data
        else:
            buf = rows
            ptr = rows.data_ptr() if hasattr(rows, "data_ptr") else rows.ctypes.data
        st = self._L.sge_enumerate(self._h, target, pattern, ptr, cap_rows, ctypes.byref(r))
        if st not in allow:
            self._check(st, "sge_enumerate")
        res = Result.of(st, r)
        if rows is None:
            nr = min(res.matches, cap_rows) if k else 0
            return res, buf[:nr, :k]
        return res, buf

    def batch_run(self, jobs, allow=(OK,)):
        """jobs: iterable of (target, pattern, mode, labelled), or an array from
        ``job_array``.  Returns (status, BatchResults)."""
        arr = job_array(jobs)
        res = np.zeros(max(len(arr), 1), dtype=RESULT_DTYPE)
        st = self._L.sge_batch_run(self._h, len(arr), arr.ctypes.data if len(arr) else None, res.ctypes.data)
        if st not in allow:
            self._check(st, "sge_batch_run")
        return st, BatchResults(st, res[:len(arr)])

    def serve_start(self, slots: int, arena_bytes: int):
        self._check(self._L.sge_serve_start(self._h, slots, arena_bytes), "sge_serve_start")

    def serve_submit(self, target: int, pattern: int, mode: int, labelled: bool):
        """Returns a ticket, or None when the query is not admissible now."""
        j = c_job(target, pattern, mode, int(bool(labelled)))
        t = ctypes.c_uint64()
        st = self._L.sge_serve_submit(self._h, ctypes.byref(j), ctypes.byref(t))
        if st == E_BUSY:
            return None
        self._check(st, "sge_serve_submit")
        return t.value

    def serve_poll(self, ticket: int):
        """Returns None while running, else the Result (status may be E_ABORTED)."""
        r = c_result()
        st = self._L.sge_serve_poll(self._h, ticket, ctypes.byref(r))
        if st == E_BUSY:
            return None
        if st not in (OK, E_ABORTED):
            self._check(st, "sge_serve_poll")
        return Result.of(st, r)

    def serve_stop(self):
        self._check(self._L.sge_serve_stop(self._h), "sge_serve_stop")
