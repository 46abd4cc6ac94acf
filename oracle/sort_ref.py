"""ctypes front of ``liboracle.so`` (see oracle_sort.c for the definitions)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.SO):
            _build.build()
        L = ctypes.CDLL(_build.SO)
        L.oracle_sort.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_sort_threads.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32]
        L.oracle_digit_histogram.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_uint32, _u64p]
        L.oracle_partition.argtypes = [_u8p, _u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_sort_segments.argtypes = [_u8p, _u64p, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32]
        L.oracle_count_runs.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u8p, _u64p,
                                        _u64p]
        for f in (L.oracle_sort, L.oracle_sort_threads, L.oracle_digit_histogram,
                  L.oracle_partition, L.oracle_sort_segments, L.oracle_count_runs):
            f.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _as_records(rec: np.ndarray) -> np.ndarray:
    rec = np.ascontiguousarray(rec, dtype=np.uint8)
    if rec.ndim != 2:
        raise ValueError("records must be a 2-D uint8 array (n, rec_bytes)")
    return rec


def _p(a: np.ndarray):
    return a.ctypes.data_as(_u8p)


def sort(rec: np.ndarray, key_bytes: int) -> np.ndarray:
    """Stable ascending sort by the little-endian key; returns a new array."""
    out = _as_records(rec).copy()
    n, r = out.shape
    if lib().oracle_sort(_p(out), n, r, key_bytes) != 0:
        raise ValueError("oracle_sort rejected the arguments")
    return out


def sort_threads(rec: np.ndarray, key_bytes: int, threads: int) -> np.ndarray:
    out = _as_records(rec).copy()
    n, r = out.shape
    if lib().oracle_sort_threads(_p(out), n, r, key_bytes, threads) != 0:
        raise ValueError("oracle_sort_threads rejected the arguments")
    return out


def sort_inplace(rec: np.ndarray, key_bytes: int, threads: int = 1) -> None:
    """Sort a C-contiguous (n, r) uint8 array in place (used for timing)."""
    n, r = rec.shape
    if lib().oracle_sort_threads(_p(rec), n, r, key_bytes, threads) != 0:
        raise ValueError("oracle_sort_threads rejected the arguments")


def sort_segments(rec: np.ndarray, offsets: np.ndarray, key_bytes: int) -> np.ndarray:
    out = _as_records(rec).copy()
    n, r = out.shape
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if int(off[-1]) != n:
        raise ValueError("offsets must end at n")
    if lib().oracle_sort_segments(_p(out), off.ctypes.data_as(_u64p), len(off) - 1, r,
                                  key_bytes) != 0:
        raise ValueError("oracle_sort_segments rejected the arguments")
    return out


def partition(rec: np.ndarray, key_bytes: int, shift: int, bits: int) -> np.ndarray:
    src = _as_records(rec)
    out = np.empty_like(src)
    n, r = src.shape
    if lib().oracle_partition(_p(src), _p(out), n, r, key_bytes, shift, bits) != 0:
        raise ValueError("oracle_partition rejected the arguments")
    return out


def digit_histogram(rec: np.ndarray, key_bytes: int, shift: int, bits: int) -> np.ndarray:
    src = _as_records(rec)
    n, r = src.shape
    cnt = np.zeros(1 << bits, dtype=np.uint64)
    if lib().oracle_digit_histogram(_p(src), n, r, key_bytes, shift, bits,
                                    cnt.ctypes.data_as(_u64p)) != 0:
        raise ValueError("oracle_digit_histogram rejected the arguments")
    return cnt


def count_runs(sorted_rec: np.ndarray, key_bytes: int):
    """Runs of equal keys in key-ordered records: (first record of each run,
    run lengths as uint64), both in key order."""
    src = _as_records(sorted_rec)
    n, r = src.shape
    uniq = np.empty_like(src)
    counts = np.empty(n, dtype=np.uint64)
    u = np.zeros(1, dtype=np.uint64)
    if lib().oracle_count_runs(_p(src), n, r, key_bytes, _p(uniq), counts.ctypes.data_as(_u64p),
                               u.ctypes.data_as(_u64p)) != 0:
        raise ValueError("oracle_count_runs rejected the arguments")
    m = int(u[0])
    return uniq[:m].copy(), counts[:m].copy()


def sort_count(rec: np.ndarray, key_bytes: int):
    """Stable sort, then duplicate removal with counts (k-mer counting, Sec. 5)."""
    return count_runs(sort(rec, key_bytes), key_bytes)
