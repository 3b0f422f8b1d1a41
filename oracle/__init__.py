"""CPU oracle for all-pairs r-NN by randomly transformed grids (RTG).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark load this package; the GPU library never does.  The
arithmetic lives in ``rtg_oracle.c`` (plain C, FP64, no FMA contraction); this
module only marshals numpy arrays through ctypes.  See ``rtg_oracle.h`` for
what each function follows in the paper.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB_PATH, build

OK, EINVAL, ENOMEM, ERANGE = 0, -1, -2, -3
NO_ROTATE, UPPER_ONLY = 1, 2
ROBOTS_SHIFT = 8


def robots(b: int) -> int:
    """Flag bits selecting the MR-metric over b robots (Sec. IV-C)."""
    return int(b) << ROBOTS_SHIFT

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


class _Result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32))]


def lib() -> ctypes.CDLL:
    """Load the oracle library, building it first if it has not been built."""
    global _lib
    if _lib is None:
        src = [os.path.join(os.path.dirname(LIB_PATH), f) for f in ("rtg_oracle.c", "rtg_oracle.h")]
        if not os.path.exists(LIB_PATH) or max(map(os.path.getmtime, src)) > os.path.getmtime(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        f64p = ctypes.POINTER(ctypes.c_double)
        f32p = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        resp = ctypes.POINTER(ctypes.POINTER(_Result))
        L.oracle_splitmix64_next.argtypes = [u64p]
        L.oracle_splitmix64_next.restype = ctypes.c_uint64
        L.oracle_uniform01.argtypes = [u64p]
        L.oracle_uniform01.restype = ctypes.c_double
        L.oracle_gaussian_pair.argtypes = [u64p, f64p, f64p]
        L.oracle_gaussian_pair.restype = None
        L.oracle_make_transforms.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint32, f64p, f64p]
        L.oracle_cell_coords.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f64p, f64p,
                                         ctypes.c_double, i64p]
        L.oracle_transform_pairs.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, f64p, f64p,
                                             ctypes.POINTER(i64p), i64p]
        L.oracle_rtg_with_transforms.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                                 f64p, f64p, ctypes.c_uint32, resp]
        L.oracle_rtg.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.c_uint32, resp]
        L.oracle_rtg_rows.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_double, f64p, f64p,
                                      ctypes.c_uint32, i64p, ctypes.c_int64, resp]
        L.oracle_bruteforce.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_uint32, resp]
        L.oracle_rtg_query.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f32p, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_double, f64p,
                                       f64p, ctypes.c_uint32, resp]
        L.oracle_result_free.argtypes = [ctypes.POINTER(_Result)]
        L.oracle_result_free.restype = None
        L.oracle_free.argtypes = [ctypes.c_void_p]
        L.oracle_free.restype = None
        for name in ("oracle_make_transforms", "oracle_cell_coords", "oracle_transform_pairs",
                     "oracle_rtg_with_transforms", "oracle_rtg", "oracle_rtg_rows",
                     "oracle_bruteforce", "oracle_rtg_query"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _points(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    return p


@dataclass
class CSR:
    """Symmetric neighbour list: row i's neighbours are col[row_ptr[i]:row_ptr[i+1]]."""
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1

    def upper_pairs(self) -> np.ndarray:
        """The unordered pairs (i<j) as an int64 [U, 2] array sorted by (i, j)."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col.astype(np.int64)
        keep = cols > rows
        return np.stack([rows[keep], cols[keep]], axis=1)


def _take_result(res_p) -> CSR:
    res = res_p.contents
    n, nnz = int(res.n), int(res.nnz)
    row_ptr = np.ctypeslib.as_array(res.row_ptr, shape=(n + 1,)).copy()
    col = (np.ctypeslib.as_array(res.col, shape=(nnz,)).copy() if nnz > 0
           else np.zeros(0, dtype=np.int32))
    lib().oracle_result_free(res_p)
    return CSR(row_ptr, col)


class SplitMix64:
    """The oracle's SplitMix64 stream (state advanced in C)."""

    def __init__(self, seed: int):
        self.state = ctypes.c_uint64(seed & (2**64 - 1))

    def next(self) -> int:
        return int(lib().oracle_splitmix64_next(ctypes.byref(self.state)))

    def uniform01(self) -> float:
        return float(lib().oracle_uniform01(ctypes.byref(self.state)))

    def gaussian_pair(self) -> tuple[float, float]:
        a, b = ctypes.c_double(), ctypes.c_double()
        lib().oracle_gaussian_pair(ctypes.byref(self.state), ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value


def make_transforms(seed: int, k: int, d: int, flags: int = 0):
    """(R [k,d,d], u [k,d]) float64: the k seeded rotations and shifts."""
    R = np.zeros((k, d, d), dtype=np.float64)
    u = np.zeros((k, d), dtype=np.float64)
    rc = lib().oracle_make_transforms(seed & (2**64 - 1), k, d, flags,
                                      _ptr(R, ctypes.c_double), _ptr(u, ctypes.c_double))
    if rc != OK:
        raise OracleError(rc, "oracle_make_transforms")
    return R, u


def cell_coords(points, R_t, u_t, inv_c: float) -> np.ndarray:
    """int64 [n, d] cell vectors floor((R p) * inv_c + u) of every point under one transform."""
    p = _points(points)
    n, d = p.shape
    R_t = np.ascontiguousarray(R_t, dtype=np.float64)
    u_t = np.ascontiguousarray(u_t, dtype=np.float64)
    kap = np.zeros((n, d), dtype=np.int64)
    rc = lib().oracle_cell_coords(_ptr(p, ctypes.c_float), n, d, _ptr(R_t, ctypes.c_double),
                                  _ptr(u_t, ctypes.c_double), float(inv_c),
                                  _ptr(kap, ctypes.c_int64))
    if rc != OK:
        raise OracleError(rc, "oracle_cell_coords")
    return kap


def transform_pairs(points, r: float, alpha: float, R_t, u_t) -> np.ndarray:
    """int64 [P, 2] pairs (i<j) that one grid reports, sorted by (i, j)."""
    p = _points(points)
    n, d = p.shape
    R_t = np.ascontiguousarray(R_t, dtype=np.float64)
    u_t = np.ascontiguousarray(u_t, dtype=np.float64)
    out = ctypes.POINTER(ctypes.c_int64)()
    cnt = ctypes.c_int64(0)
    rc = lib().oracle_transform_pairs(_ptr(p, ctypes.c_float), n, d, float(r), float(alpha),
                                      _ptr(R_t, ctypes.c_double), _ptr(u_t, ctypes.c_double),
                                      ctypes.byref(out), ctypes.byref(cnt))
    if rc != OK:
        raise OracleError(rc, "oracle_transform_pairs")
    m = int(cnt.value)
    pairs = (np.ctypeslib.as_array(out, shape=(m, 2)).copy() if m > 0
             else np.zeros((0, 2), dtype=np.int64))
    lib().oracle_free(ctypes.cast(out, ctypes.c_void_p))
    return pairs


def rtg_with_transforms(points, r: float, alpha: float, R, u, flags: int = 0) -> CSR:
    p = _points(points)
    n, d = p.shape
    R = np.ascontiguousarray(R, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    k = R.shape[0]
    if R.shape != (k, d, d) or u.shape != (k, d):
        raise ValueError("R must be [k,d,d] and u [k,d]")
    res = ctypes.POINTER(_Result)()
    rc = lib().oracle_rtg_with_transforms(_ptr(p, ctypes.c_float), n, d, float(r), k, float(alpha),
                                          _ptr(R, ctypes.c_double), _ptr(u, ctypes.c_double),
                                          flags, ctypes.byref(res))
    if rc != OK:
        raise OracleError(rc, "oracle_rtg_with_transforms")
    return _take_result(res)


def rtg(points, r: float, k: int, alpha: float, seed: int, flags: int = 0) -> CSR:
    p = _points(points)
    n, d = p.shape
    res = ctypes.POINTER(_Result)()
    rc = lib().oracle_rtg(_ptr(p, ctypes.c_float), n, d, float(r), int(k), float(alpha),
                          seed & (2**64 - 1), flags, ctypes.byref(res))
    if rc != OK:
        raise OracleError(rc, "oracle_rtg")
    return _take_result(res)


def rtg_rows(points, r: float, alpha: float, R, u, rows, flags: int = 0) -> list[np.ndarray]:
    """Neighbour lists (ascending int32) of the given rows of the symmetric RTG
    output, each computed on its own (flags: robots(b) for the MR-metric)."""
    p = _points(points)
    n, d = p.shape
    R = np.ascontiguousarray(R, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    k = R.shape[0]
    if R.shape != (k, d, d) or u.shape != (k, d):
        raise ValueError("R must be [k,d,d] and u [k,d]")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    res = ctypes.POINTER(_Result)()
    rc = lib().oracle_rtg_rows(_ptr(p, ctypes.c_float), n, d, float(r), k, float(alpha),
                               _ptr(R, ctypes.c_double), _ptr(u, ctypes.c_double), flags,
                               _ptr(rows, ctypes.c_int64), len(rows), ctypes.byref(res))
    if rc != OK:
        raise OracleError(rc, "oracle_rtg_rows")
    csr = _take_result(res)
    return [csr.col[csr.row_ptr[s]:csr.row_ptr[s + 1]] for s in range(len(rows))]


def rtg_query(points, queries, r: float, alpha: float, R, u, flags: int = 0) -> CSR:
    """Query mode: row s lists the indexed points within r of queries[s] that
    share a cell with it under some transform (ascending, once each); flags:
    robots(b) for the MR-metric."""
    p = _points(points)
    q = _points(queries)
    n, d = p.shape
    if q.shape[1] != d:
        raise ValueError("queries must have the points' dimension")
    R = np.ascontiguousarray(R, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    k = R.shape[0]
    if R.shape != (k, d, d) or u.shape != (k, d):
        raise ValueError("R must be [k,d,d] and u [k,d]")
    res = ctypes.POINTER(_Result)()
    rc = lib().oracle_rtg_query(_ptr(p, ctypes.c_float), n, d, _ptr(q, ctypes.c_float), len(q),
                                float(r), k, float(alpha), _ptr(R, ctypes.c_double),
                                _ptr(u, ctypes.c_double), flags, ctypes.byref(res))
    if rc != OK:
        raise OracleError(rc, "oracle_rtg_query")
    return _take_result(res)


def bruteforce(points, r: float, flags: int = 0) -> CSR:
    p = _points(points)
    n, d = p.shape
    res = ctypes.POINTER(_Result)()
    rc = lib().oracle_bruteforce(_ptr(p, ctypes.c_float), n, d, float(r), flags, ctypes.byref(res))
    if rc != OK:
        raise OracleError(rc, "oracle_bruteforce")
    return _take_result(res)
