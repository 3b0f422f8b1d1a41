"""Thin Python binding of the RTG library (include/rtg.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of librtg.so.  PyTorch supplies device memory (the context's arena is
one torch tensor) and the HIP stream; results come back as zero-copy torch
views into that arena, valid until released.

The library must be built (``paper_1409_8112_amd/build.py``); if it is
missing it is built on first use.  There is no CPU fallback: without the
library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from . import build as _build

OK, EAGAIN, EINVAL, ENOMEM, ERANGE, EDEVICE, ENOENT = 0, 1, -1, -2, -3, -4, -5
NO_ROTATE, UPPER_ONLY, DEDUP_SORT, DEDUP_BITMAP = 1, 2, 4, 8
ROBOTS_SHIFT = 8


def robots(b: int) -> int:
    """Flag bits of the MR-metric over b robots (RTG_ROBOTS(b))."""
    return int(b) << ROBOTS_SHIFT
# kernel ids of rtg_stats.kernel_* (RTG_K_* in rtg.h)
KERNELS = ["stage", "keys", "key_hist", "key_scatter", "cells", "pairs", "pair_hist",
           "pair_scatter", "unique", "csr", "scan", "gather", "compact"]
NKERNELS = len(KERNELS)
TIME_PHASES = 1 << 31

_lib = None
_lib_lock = threading.Lock()


class RTGError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class rtg_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("handle", ctypes.c_uint64), ("pairs", ctypes.c_int64)]


class rtg_query(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("r", ctypes.c_double), ("k", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


class rtg_tuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "d", "log2_points", "tests_per_wave", "unit_tiles", "part_threads", "bucket_blocks",
        "bucket_entries", "sort")] + [("ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class rtg_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "d", "k", "point_transforms", "cells", "tests", "candidates", "band_rechecks",
        "unique_pairs")] + [(name, ctypes.c_int32) for name in (
            "key_bits", "key_passes", "pair_bits", "transforms_per_sort")] + [
        (name, ctypes.c_double) for name in (
            "ms_stage", "ms_keys", "ms_key_sort", "ms_cells", "ms_pairs", "ms_pair_sort",
            "ms_unique", "ms_csr", "ms_total")] + [
        ("kernel_launches", ctypes.c_int64 * NKERNELS),
        ("kernel_bytes", ctypes.c_double * NKERNELS),
        ("kernel_ms", ctypes.c_double * NKERNELS),
        ("served_requests", ctypes.c_int64), ("served_batches", ctypes.c_int64),
        ("matrix_screen_launches", ctypes.c_int64), ("served_small", ctypes.c_int64)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name.startswith("kernel_") else v
        return out


def lib() -> ctypes.CDLL:
    """Load librtg.so (building it if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_build.LIB_PATH):
                _build.build()
            L = ctypes.CDLL(_build.LIB_PATH)
            vp, i64, i32, u64, u32, f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double)
            sig = {
                "rtg_create": [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t, vp],
                "rtg_destroy": [vp],
                "rtg_all_pairs": [vp, vp, i64, i32, f64, i32, f64, u64, u32,
                                  ctypes.POINTER(rtg_csr)],
                "rtg_all_pairs_with_transforms": [vp, vp, i64, i32, f64, i32, f64, vp, vp, u32,
                                                  ctypes.POINTER(rtg_csr)],
                "rtg_all_pairs_noalloc": [vp, vp, i64, i32, f64, i32, f64, u64, u32, vp, vp,
                                          i64, ctypes.POINTER(i64)],
                "rtg_all_pairs_batched": [vp, ctypes.POINTER(rtg_query), i32,
                                          ctypes.POINTER(rtg_csr)],
                "rtg_plan_create": [vp, ctypes.POINTER(rtg_query), i32, ctypes.POINTER(vp)],
                "rtg_plan_run": [vp, ctypes.POINTER(rtg_query), i32, ctypes.POINTER(rtg_csr)],
                "rtg_plan_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(i64)],
                "rtg_plan_destroy": [vp],
                "rtg_submit": [vp, ctypes.POINTER(rtg_query), ctypes.POINTER(u64)],
                "rtg_poll": [vp, u64, ctypes.POINTER(rtg_csr)],
                "rtg_release": [vp, u64],
                "rtg_release_many": [vp, ctypes.POINTER(u64), i32],
                "rtg_make_transforms": [u64, i32, i32, u32, vp, vp],
                "rtg_choose_params": [i32, f64, f64, u32, ctypes.POINTER(i32),
                                      ctypes.POINTER(f64), ctypes.POINTER(f64)],
                "rtg_model_recall": [i32, i32, f64, u32, ctypes.POINTER(f64)],
                "rtg_index_build": [vp, vp, i64, i32, f64, i32, f64, u64, u32,
                                    ctypes.POINTER(u64)],
                "rtg_index_query": [vp, u64, vp, i64, ctypes.POINTER(rtg_csr)],
                "rtg_autotune": [vp, ctypes.POINTER(rtg_query), i32, i32,
                                 ctypes.POINTER(rtg_tuning)],
                "rtg_set_tuning": [vp, ctypes.POINTER(rtg_tuning)],
                "rtg_get_tuning": [vp, i32, i64, ctypes.POINTER(rtg_tuning)],
                "rtg_save_tuning": [vp, ctypes.c_char_p],
                "rtg_load_tuning": [vp, ctypes.c_char_p],
                "rtg_tune_params": [vp, vp, i64, i32, f64, f64, u32, i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(f64), ctypes.POINTER(f64), ctypes.POINTER(f64)],
                "rtg_set_timing": [vp, u32],
                "rtg_get_stats": [vp, ctypes.POINTER(rtg_stats)],
                "rtg_debug_cell_coords": [vp, vp, i64, i32, f64, f64, vp, vp, vp],
            }
            for name, args in sig.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            L.rtg_strerror.argtypes = [ctypes.c_int]
            L.rtg_strerror.restype = ctypes.c_char_p
            _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().rtg_strerror(code).decode()


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise RTGError(rc, what)


def rtg_make_transforms(seed: int, k: int, d: int, flags: int = 0):
    """(R [k,d,d], u [k,d]) float64, the library's seeded transforms."""
    R = np.zeros((k, d, d), dtype=np.float64)
    u = np.zeros((k, d), dtype=np.float64)
    _check(lib().rtg_make_transforms(seed & (2**64 - 1), k, d, flags, R.ctypes.data,
                                     u.ctypes.data), "rtg_make_transforms")
    return R, u


make_transforms = rtg_make_transforms


def choose_params(d: int, target_recall: float, mean_neighbours: float, flags: int = 0):
    """(k, alpha, modelled recall) of least modelled cost reaching the target."""
    k, a, rc = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(lib().rtg_choose_params(int(d), float(target_recall), float(mean_neighbours), flags,
                                   ctypes.byref(k), ctypes.byref(a), ctypes.byref(rc)),
           "rtg_choose_params")
    return int(k.value), float(a.value), float(rc.value)


def model_recall(d: int, k: int, alpha: float, flags: int = 0) -> float:
    """The modelled recall of k grids of cell factor alpha in dimension d."""
    rc = ctypes.c_double()
    _check(lib().rtg_model_recall(int(d), int(k), float(alpha), flags, ctypes.byref(rc)),
           "rtg_model_recall")
    return float(rc.value)


class Result:
    """A device-resident neighbour list: row_ptr (torch.int64 [n+1]) and col
    (torch.int32 [nnz]) are views into the context's arena, made on first
    use, valid until release()."""

    __slots__ = ("ctx", "handle", "n", "nnz", "pairs", "released", "_rp_ptr", "_col_ptr",
                 "_row_ptr", "_col")

    def __init__(self, ctx: "Context", handle: int, n: int, nnz: int, pairs: int,
                 rp_ptr: int, col_ptr: int):
        self.ctx, self.handle, self.n, self.nnz, self.pairs = ctx, handle, n, nnz, pairs
        self.released = False
        self._rp_ptr, self._col_ptr = rp_ptr, col_ptr
        self._row_ptr = self._col = None

    @property
    def row_ptr(self):
        if self._row_ptr is None:
            self._row_ptr = self.ctx._view(self._rp_ptr, self.n + 1, self.ctx.torch.int64)
        return self._row_ptr

    @property
    def col(self):
        if self._col is None:
            self._col = self.ctx._view(self._col_ptr, self.nnz, self.ctx.torch.int32)
        return self._col

    def to_numpy(self):
        return self.row_ptr.cpu().numpy().copy(), self.col.cpu().numpy().copy()

    def release(self) -> None:
        if not self.released:
            self.ctx.rtg_release(self.handle)
            self.released = True


class Plan:
    """A plan of one context (rtg_plan_*): run() returns what
    rtg_all_pairs_batched returns for the same queries."""

    def __init__(self, ctx: "Context", handle, nq: int):
        self.ctx, self.h, self.nq = ctx, handle, nq

    def run(self, queries) -> list[Result]:
        if self.h is None:
            raise RTGError(EINVAL, "plan destroyed")
        nq = len(queries)
        qs, _pts = self.ctx._query_table(queries)
        outs = (rtg_csr * max(nq, 1))()
        _check(lib().rtg_plan_run(self.h, qs.ctypes.data_as(ctypes.POINTER(rtg_query)), nq, outs),
               "rtg_plan_run")
        return self.ctx._results(outs, nq)

    def info(self) -> dict:
        c, r, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().rtg_plan_info(self.h, ctypes.byref(c), ctypes.byref(r), ctypes.byref(w)),
               "rtg_plan_info")
        return {"captures": c.value, "replays": r.value, "workspace_bytes": w.value}

    def destroy(self) -> None:
        if self.h is not None and self.ctx.h.value:
            _check(lib().rtg_plan_destroy(self.h), "rtg_plan_destroy")
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


class Context:
    """An RTG context on one GPU: an arena of `arena_bytes` device memory from
    torch and torch's current HIP stream."""

    def __init__(self, device: int = 0, arena_bytes: int | None = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("RTG needs a ROCm GPU; none is visible")
        self.torch = torch
        self.device = device
        with torch.cuda.device(device):
            if arena_bytes is None:
                free, _ = torch.cuda.mem_get_info(device)
                arena_bytes = int(min(64 << 30, free * 0.6))
            self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
            self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.arena_base = self.arena.data_ptr()
        self.arena_bytes = arena_bytes
        h = ctypes.c_void_p()
        _check(lib().rtg_create(ctypes.byref(h), device, ctypes.c_void_p(self.arena_base),
                                arena_bytes, ctypes.c_void_p(self.stream.cuda_stream)),
               "rtg_create")
        self.h = h

    # -- lifetime --------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value:
            for p in getattr(self, "_plans", []):
                p.destroy()  # a plan goes before its context
            lib().rtg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- results -----------------------------------------------------------------
    def _view(self, ptr: int, count: int, dtype):
        t = self.torch
        if count == 0:
            return t.empty(0, dtype=dtype, device=self.arena.device)
        off = ptr - self.arena_base
        nbytes = count * t.empty(0, dtype=dtype).element_size()
        if off < 0 or off + nbytes > self.arena_bytes:
            raise RuntimeError("result outside the arena")
        return self.arena[off:off + nbytes].view(dtype)

    def _result(self, c: rtg_csr) -> Result:
        return Result(self, int(c.handle), int(c.n), int(c.nnz), int(c.pairs), int(c.row_ptr),
                      int(c.col or 0))

    def _points(self, points):
        if points.dtype != self.torch.float32:
            raise TypeError("points must be a float32 tensor")
        if points.dim() != 2 or not points.is_cuda or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, d] CUDA tensor")
        return points

    # -- calls -------------------------------------------------------------------
    def rtg_all_pairs(self, points, r: float, k: int, alpha: float, seed: int,
                      flags: int = 0) -> Result:
        p = self._points(points)
        out = rtg_csr()
        _check(lib().rtg_all_pairs(self.h, p.data_ptr(), p.shape[0], p.shape[1], float(r), int(k),
                                   float(alpha), seed & (2**64 - 1), flags, ctypes.byref(out)),
               "rtg_all_pairs")
        return self._result(out)

    def rtg_all_pairs_noalloc(self, points, r: float, k: int, alpha: float, seed: int,
                              row_ptr, col, flags: int = 0) -> int:
        """rtg_all_pairs into caller tensors (row_ptr int64 [n+1], col int32
        [capacity]) with no device allocation; returns nnz.  Raises RTGError
        (ENOMEM) when col is too small, with the entries needed in .needed."""
        p = self._points(points)
        t = self.torch
        if row_ptr.dtype != t.int64 or col.dtype != t.int32:
            raise TypeError("row_ptr must be int64 and col int32")
        if not (row_ptr.is_cuda and col.is_cuda and row_ptr.is_contiguous() and
                col.is_contiguous()) or row_ptr.numel() != p.shape[0] + 1:
            raise ValueError("row_ptr must be a contiguous CUDA tensor of n+1 entries and col "
                             "a contiguous CUDA tensor")
        nnz = ctypes.c_int64(0)
        rc = lib().rtg_all_pairs_noalloc(self.h, p.data_ptr(), p.shape[0], p.shape[1], float(r),
                                         int(k), float(alpha), seed & (2**64 - 1), flags,
                                         row_ptr.data_ptr(),
                                         col.data_ptr() if col.numel() else None, col.numel(),
                                         ctypes.byref(nnz))
        if rc == ENOMEM:
            err = RTGError(rc, "rtg_all_pairs_noalloc")
            err.needed = int(nnz.value)
            raise err
        _check(rc, "rtg_all_pairs_noalloc")
        return int(nnz.value)

    def rtg_all_pairs_with_transforms(self, points, r: float, alpha: float, R, u,
                                      flags: int = 0) -> Result:
        p = self._points(points)
        R = np.ascontiguousarray(R, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        k, d = R.shape[0], p.shape[1]
        if R.shape != (k, d, d) or u.shape != (k, d):
            raise ValueError("R must be [k,d,d] and u [k,d]")
        out = rtg_csr()
        _check(lib().rtg_all_pairs_with_transforms(self.h, p.data_ptr(), p.shape[0], d, float(r), k,
                                                   float(alpha), R.ctypes.data, u.ctypes.data,
                                                   flags, ctypes.byref(out)),
               "rtg_all_pairs_with_transforms")
        return self._result(out)

    def _query_table(self, queries):
        nq = len(queries)
        qs = np.zeros(max(nq, 1), dtype=np.dtype(rtg_query))
        pts = [self._points(q["points"]) for q in queries]
        if nq:
            qs["points"][:nq] = [p.data_ptr() for p in pts]
            qs["n"][:nq] = [p.shape[0] for p in pts]
            qs["d"][:nq] = [p.shape[1] for p in pts]
            qs["r"][:nq] = [q["r"] for q in queries]
            qs["k"][:nq] = [q["k"] for q in queries]
            qs["alpha"][:nq] = [q["alpha"] for q in queries]
            qs["seed"][:nq] = [q.get("seed", 0) & (2**64 - 1) for q in queries]
            qs["flags"][:nq] = [q.get("flags", 0) for q in queries]
        return qs, pts

    def rtg_autotune(self, queries, reps: int = 3) -> dict:
        """Tunes the launch settings for these queries (one dimension) and
        installs them; returns the entry (rtg_tuning) as a dict."""
        qs, _pts = self._query_table(queries)
        out = rtg_tuning()
        _check(lib().rtg_autotune(self.h, qs.ctypes.data_as(ctypes.POINTER(rtg_query)),
                                  len(queries), int(reps), ctypes.byref(out)), "rtg_autotune")
        return out.as_dict()

    def rtg_set_tuning(self, entry: dict) -> None:
        t = rtg_tuning(**{k: v for k, v in entry.items() if k in dict(rtg_tuning._fields_)})
        _check(lib().rtg_set_tuning(self.h, ctypes.byref(t)), "rtg_set_tuning")

    def rtg_get_tuning(self, d: int, points: int) -> dict:
        out = rtg_tuning()
        _check(lib().rtg_get_tuning(self.h, int(d), int(points), ctypes.byref(out)),
               "rtg_get_tuning")
        return out.as_dict()

    def rtg_save_tuning(self, path: str) -> None:
        _check(lib().rtg_save_tuning(self.h, os.fsencode(path)), "rtg_save_tuning")

    def rtg_load_tuning(self, path: str) -> None:
        _check(lib().rtg_load_tuning(self.h, os.fsencode(path)), "rtg_load_tuning")

    def rtg_tune_params(self, points, r: float, target_recall: float, flags: int = 0,
                        reps: int = 2):
        """(k, alpha, modelled recall, ms): the fastest measured parameters
        whose modelled recall reaches the target."""
        p = self._points(points)
        k, a, rec, ms = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().rtg_tune_params(self.h, p.data_ptr(), p.shape[0], p.shape[1], float(r),
                                     float(target_recall), flags, int(reps), ctypes.byref(k),
                                     ctypes.byref(a), ctypes.byref(rec), ctypes.byref(ms)),
               "rtg_tune_params")
        return int(k.value), float(a.value), float(rec.value), float(ms.value)

    def _results(self, outs, nq: int) -> list[Result]:
        if nq == 0:
            return []
        # the output table read column by column (one numpy pass per field)
        arr = np.frombuffer(outs, dtype=np.dtype(rtg_csr), count=nq)
        cols = [arr[f].tolist() for f in ("handle", "n", "nnz", "pairs", "row_ptr", "col")]
        return [Result(self, *t) for t in zip(*cols)]

    def rtg_all_pairs_batched(self, queries) -> list[Result]:
        """queries: list of dicts with points, r, k, alpha, seed, flags."""
        nq = len(queries)
        # the query table filled column by column (one numpy write per field)
        qs, _pts = self._query_table(queries)
        outs = (rtg_csr * max(nq, 1))()
        _check(lib().rtg_all_pairs_batched(self.h, qs.ctypes.data_as(ctypes.POINTER(rtg_query)),
                                           nq, outs), "rtg_all_pairs_batched")
        return self._results(outs, nq)

    def rtg_plan_create(self, queries) -> "Plan":
        """A plan for repeated batched calls of these queries' shape (each
        query's n, d, k and flags)."""
        qs, _pts = self._query_table(queries)
        h = ctypes.c_void_p()
        _check(lib().rtg_plan_create(self.h, qs.ctypes.data_as(ctypes.POINTER(rtg_query)),
                                     len(queries), ctypes.byref(h)), "rtg_plan_create")
        plan = Plan(self, h, len(queries))
        if not hasattr(self, "_plans"):
            self._plans = []
        self._plans.append(plan)
        return plan

    def rtg_submit(self, points, r: float, k: int, alpha: float, seed: int,
                   flags: int = 0) -> int | None:
        """A ticket, or None when the points cannot be staged yet (retry later).
        The points are copied before this returns."""
        p = self._points(points)
        q = rtg_query(p.data_ptr(), p.shape[0], p.shape[1], float(r), int(k), float(alpha),
                      seed & (2**64 - 1), flags)
        t = ctypes.c_uint64()
        rc = lib().rtg_submit(self.h, ctypes.byref(q), ctypes.byref(t))
        if rc == EAGAIN:
            return None
        _check(rc, "rtg_submit")
        return int(t.value)

    def rtg_poll(self, ticket: int):
        """The Result when done, None while pending; raises on the request's error."""
        out = rtg_csr()
        rc = lib().rtg_poll(self.h, ticket, ctypes.byref(out))
        if rc == EAGAIN:
            return None
        _check(rc, "rtg_poll")
        return self._result(out)

    def wait(self, ticket: int, timeout_s: float = 60.0, sleep_s: float = 1e-4):
        """Poll until the request is done (raises TimeoutError after timeout_s)."""
        import time
        t_end = time.monotonic() + timeout_s
        while True:
            res = self.rtg_poll(ticket)
            if res is not None:
                return res
            if time.monotonic() > t_end:
                raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
            time.sleep(sleep_s)

    def rtg_release(self, handle: int) -> None:
        _check(lib().rtg_release(self.h, handle), "rtg_release")

    def rtg_release_many(self, results) -> None:
        """Release every not yet released Result of the list in one call."""
        todo = [r for r in results if not r.released]
        if not todo:
            return
        hs = np.array([r.handle for r in todo], dtype=np.uint64)
        rc = lib().rtg_release_many(self.h, hs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    len(hs))
        for r in todo:
            r.released = True
        _check(rc, "rtg_release_many")

    def rtg_index_build(self, points, r: float, k: int, alpha: float, seed: int,
                        flags: int = 0) -> int:
        """Sorts the k grids of `points` once and keeps them; returns the index
        handle (free with release)."""
        p = self._points(points)
        h = ctypes.c_uint64()
        _check(lib().rtg_index_build(self.h, p.data_ptr(), p.shape[0], p.shape[1], float(r),
                                     int(k), float(alpha), seed & (2**64 - 1), flags,
                                     ctypes.byref(h)), "rtg_index_build")
        return int(h.value)

    def rtg_index_query(self, index: int, queries) -> Result:
        """Row s: the indexed points within r of queries[s] sharing a cell with it
        under some grid (ascending)."""
        q = self._points(queries)
        out = rtg_csr()
        _check(lib().rtg_index_query(self.h, index, q.data_ptr(), q.shape[0], ctypes.byref(out)),
               "rtg_index_query")
        return self._result(out)

    def rtg_set_timing(self, mask: int) -> None:
        """Bit i times kernel id i (KERNELS[i]); TIME_PHASES times the phases."""
        _check(lib().rtg_set_timing(self.h, int(mask) & 0xFFFFFFFF), "rtg_set_timing")

    def rtg_get_stats(self) -> dict:
        s = rtg_stats()
        _check(lib().rtg_get_stats(self.h, ctypes.byref(s)), "rtg_get_stats")
        return s.as_dict()

    def rtg_debug_cell_coords(self, points, r: float, alpha: float, R_t, u_t) -> np.ndarray:
        p = self._points(points)
        n, d = p.shape
        R_t = np.ascontiguousarray(R_t, dtype=np.float64)
        u_t = np.ascontiguousarray(u_t, dtype=np.float64)
        kap = np.zeros((n, d), dtype=np.int64)
        _check(lib().rtg_debug_cell_coords(self.h, p.data_ptr(), n, d, float(r), float(alpha),
                                           R_t.ctypes.data, u_t.ctypes.data, kap.ctypes.data),
               "rtg_debug_cell_coords")
        return kap

    # short aliases
    index_build = rtg_index_build
    index_query = rtg_index_query
    all_pairs = rtg_all_pairs
    all_pairs_noalloc = rtg_all_pairs_noalloc
    autotune = rtg_autotune
    set_tuning = rtg_set_tuning
    get_tuning = rtg_get_tuning
    save_tuning = rtg_save_tuning
    load_tuning = rtg_load_tuning
    tune_params = rtg_tune_params
    all_pairs_with_transforms = rtg_all_pairs_with_transforms
    all_pairs_batched = rtg_all_pairs_batched
    plan_create = rtg_plan_create
    release_many = rtg_release_many
    submit = rtg_submit
    poll = rtg_poll
    release = rtg_release
    set_timing = rtg_set_timing
    stats = rtg_get_stats
    debug_cell_coords = rtg_debug_cell_coords
