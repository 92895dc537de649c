"""Plain CPU oracle for the join and group-by hot path.

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
CPU-baseline leg import this package. The GPU library never imports it.

The C part (oracle.c, built with gcc into liboracle.so) computes the plain
relational definitions with qsort and binary search. This module wraps it with
NumPy and adds the projections that turn matched row pairs into the join's
output columns.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (host only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.oracle_join_pairs.restype = i64
        L.oracle_join_pairs.argtypes = [ctypes.c_int, vp, i64, vp, i64, vp, vp, i64]
        L.oracle_rows_fingerprint.restype = None
        L.oracle_rows_fingerprint.argtypes = [vp, vp, i32, i64, vp]
        L.oracle_join_fingerprint.restype = ctypes.c_int
        L.oracle_join_fingerprint.argtypes = [ctypes.c_int, vp, i64, vp, vp, i32,
                                              vp, i64, vp, vp, i32, vp]
        L.oracle_groupby.restype = i64
        L.oracle_groupby.argtypes = [ctypes.c_int, vp, i64, vp, i32, vp, vp, vp, vp, vp]
        L.oracle_groupby64.restype = i64
        L.oracle_groupby64.argtypes = [ctypes.c_int, vp, i64, vp, i32, vp, vp, vp, vp, vp]
        L.oracle_partition.restype = ctypes.c_int
        L.oracle_partition.argtypes = [ctypes.c_int, vp, i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, vp, vp]
        L.oracle_digit_source.restype = ctypes.c_uint64
        L.oracle_digit_source.argtypes = [ctypes.c_int, i64, ctypes.c_int]
        L.oracle_hll_registers.restype = None
        L.oracle_hll_registers.argtypes = [ctypes.c_int, vp, i64, ctypes.c_int, vp]
        L.oracle_hgb_ids.restype = i64
        L.oracle_hgb_ids.argtypes = [ctypes.c_int, vp, i64, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _key_bytes(k: np.ndarray) -> int:
    if k.dtype == np.int32:
        return 4
    if k.dtype == np.int64:
        return 8
    raise TypeError(f"keys must be int32 or int64, got {k.dtype}")


def join_pairs(r_key: np.ndarray, s_key: np.ndarray):
    """Matching (R row, S row) index pairs of R |><| S, in S order then R order."""
    r_key = np.ascontiguousarray(r_key)
    s_key = np.ascontiguousarray(s_key)
    kb = _key_bytes(r_key)
    assert s_key.dtype == r_key.dtype
    L = lib()
    t = L.oracle_join_pairs(kb, _ptr(r_key), len(r_key), _ptr(s_key), len(s_key), None, None, 0)
    if t < 0:
        raise MemoryError("oracle_join_pairs")
    out_r = np.empty(t, np.int64)
    out_s = np.empty(t, np.int64)
    t2 = L.oracle_join_pairs(kb, _ptr(r_key), len(r_key), _ptr(s_key), len(s_key),
                             _ptr(out_r), _ptr(out_s), t)
    assert t2 == t
    return out_r, out_s


def join(r_key, r_pay, s_key, s_pay):
    """Materialized join output T(key, r_1.., s_1..) as a list of columns
    (Section 2.2: output columns are the key, R's payloads, then S's)."""
    ir, js = join_pairs(r_key, s_key)
    cols = [np.asarray(s_key)[js]]
    cols += [np.asarray(p)[ir] for p in r_pay]
    cols += [np.asarray(p)[js] for p in s_pay]
    return cols


def rows_fingerprint(cols) -> tuple[int, int, int]:
    """(rows, sum H(row), sum H(row)^2) mod 2^64 over a table given as columns."""
    cols = [np.ascontiguousarray(c) for c in cols]
    n = len(cols[0]) if cols else 0
    ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
    widths = np.array([c.dtype.itemsize for c in cols], np.int32)
    out = np.zeros(3, np.uint64)
    lib().oracle_rows_fingerprint(ctypes.cast(ptrs, ctypes.c_void_p), _ptr(widths),
                                  len(cols), n, _ptr(out))
    return int(out[0]), int(out[1]), int(out[2])


def join_fingerprint(r_key, r_pay, s_key, s_pay) -> tuple[int, int, int]:
    """Fingerprint of the join output without materializing it."""
    r_key = np.ascontiguousarray(r_key)
    s_key = np.ascontiguousarray(s_key)
    r_pay = [np.ascontiguousarray(p) for p in r_pay]
    s_pay = [np.ascontiguousarray(p) for p in s_pay]
    rp = (ctypes.c_void_p * max(1, len(r_pay)))(*[p.ctypes.data for p in r_pay])
    sp = (ctypes.c_void_p * max(1, len(s_pay)))(*[p.ctypes.data for p in s_pay])
    rw = np.array([p.dtype.itemsize for p in r_pay] or [4], np.int32)
    sw = np.array([p.dtype.itemsize for p in s_pay] or [4], np.int32)
    out = np.zeros(3, np.uint64)
    rc = lib().oracle_join_fingerprint(_key_bytes(r_key), _ptr(r_key), len(r_key),
                                       ctypes.cast(rp, ctypes.c_void_p), _ptr(rw), len(r_pay),
                                       _ptr(s_key), len(s_key),
                                       ctypes.cast(sp, ctypes.c_void_p), _ptr(sw), len(s_pay),
                                       _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_join_fingerprint")
    return int(out[0]), int(out[1]), int(out[2])


def groupby(keys: np.ndarray, vals) -> dict:
    """Per distinct key (ascending): count, and per value column sum/min/max.
    Any int64 value column makes every column int64 (oracle_groupby64: min and
    max come back as int64, sums modulo 2^64)."""
    keys = np.ascontiguousarray(keys)
    if any(np.asarray(v).dtype == np.int64 for v in vals):
        return _groupby64(keys, [np.ascontiguousarray(v, dtype=np.int64) for v in vals])
    vals = [np.ascontiguousarray(v, dtype=np.int32) for v in vals]
    n = len(keys)
    nv = len(vals)
    cap = max(n, 1)
    ok = np.empty(cap, np.int64)
    oc = np.empty(cap, np.int64)
    osum = np.empty(max(nv, 1) * cap, np.int64)
    omin = np.empty(max(nv, 1) * cap, np.int32)
    omax = np.empty(max(nv, 1) * cap, np.int32)
    vp = (ctypes.c_void_p * max(1, nv))(*[v.ctypes.data for v in vals])
    g = lib().oracle_groupby(_key_bytes(keys), _ptr(keys), n, ctypes.cast(vp, ctypes.c_void_p), nv,
                             _ptr(ok), _ptr(oc), _ptr(osum), _ptr(omin), _ptr(omax))
    if g < 0:
        raise MemoryError("oracle_groupby")
    kd = keys.dtype
    return {
        "key": ok[:g].astype(kd),
        "count": oc[:g].copy(),
        "sum": [osum[v * cap: v * cap + g].copy() for v in range(nv)],
        "min": [omin[v * cap: v * cap + g].copy() for v in range(nv)],
        "max": [omax[v * cap: v * cap + g].copy() for v in range(nv)],
    }


def _groupby64(keys: np.ndarray, vals) -> dict:
    n, nv = len(keys), len(vals)
    cap = max(n, 1)
    ok = np.empty(cap, np.int64)
    oc = np.empty(cap, np.int64)
    osum = np.empty(max(nv, 1) * cap, np.int64)
    omin = np.empty(max(nv, 1) * cap, np.int64)
    omax = np.empty(max(nv, 1) * cap, np.int64)
    vp = (ctypes.c_void_p * max(1, nv))(*[v.ctypes.data for v in vals])
    g = lib().oracle_groupby64(_key_bytes(keys), _ptr(keys), n, ctypes.cast(vp, ctypes.c_void_p), nv,
                               _ptr(ok), _ptr(oc), _ptr(osum), _ptr(omin), _ptr(omax))
    if g < 0:
        raise MemoryError("oracle_groupby64")
    return {
        "key": ok[:g].astype(keys.dtype),
        "count": oc[:g].copy(),
        "sum": [osum[v * cap: v * cap + g].copy() for v in range(nv)],
        "min": [omin[v * cap: v * cap + g].copy() for v in range(nv)],
        "max": [omax[v * cap: v * cap + g].copy() for v in range(nv)],
    }


DIGIT_BITS, DIGIT_HASH, DIGIT_ORDERED = 0, 1, 2


def partition(keys: np.ndarray, lo: int, bits: int, mode: int = DIGIT_BITS):
    """Stable partition by digit = bits [lo, lo+bits) of the digit source.
    Returns (perm, hist): output position i holds input row perm[i]."""
    keys = np.ascontiguousarray(keys)
    n = len(keys)
    perm = np.empty(max(n, 1), np.int64)
    hist = np.empty(1 << bits, np.int64)
    rc = lib().oracle_partition(_key_bytes(keys), _ptr(keys), n, lo, bits, mode,
                                _ptr(perm), _ptr(hist))
    if rc != 0:
        raise MemoryError("oracle_partition")
    return perm[:n], hist


def digit_source(key: int, key_bytes: int, mode: int) -> int:
    return int(lib().oracle_digit_source(key_bytes, key, mode))


def hll_registers(keys: np.ndarray, bits: int = 10) -> np.ndarray:
    """HyperLogLog registers of the keys (see oracle_hll_registers)."""
    keys = np.ascontiguousarray(keys)
    regs = np.zeros(1 << bits, np.uint32)
    lib().oracle_hll_registers(_key_bytes(keys), _ptr(keys), len(keys), bits, _ptr(regs))
    return regs


def hll_estimate(keys: np.ndarray, bits: int = 10) -> float:
    """Distinct-key estimate of Flajolet et al. (2007) from hll_registers: the
    raw estimate alpha_m m^2 / sum_j 2^-M[j] with alpha_m = 0.7213 / (1 + 1.079 / m)
    (their constant for m >= 128), replaced by linear counting m ln(m / V) when
    it is at most 5m/2 and V registers are still zero. The estimate is capped at
    the row count (a reading of ours: n rows hold at most n distinct keys); with
    no rows it is 0."""
    n = len(keys)
    if n == 0:
        return 0.0
    regs = hll_registers(keys, bits)
    m = float(1 << bits)
    raw = (0.7213 / (1.0 + 1.079 / m)) * m * m / float(np.sum(np.ldexp(1.0, -regs.astype(np.int64))))
    zeros = int(np.count_nonzero(regs == 0))
    est = m * math.log(m / zeros) if raw <= 2.5 * m and zeros > 0 else raw
    return min(est, float(n))


def varying_key_bytes(keys: np.ndarray) -> int:
    """Key bytes (of the key width) whose value differs between some two rows:
    the passes a radix sort of the raw keys cannot skip. 0 with no rows."""
    keys = np.ascontiguousarray(keys)
    if len(keys) == 0:
        return 0
    kb = _key_bytes(keys)
    b = keys.view(np.uint8).reshape(len(keys), kb)
    return int(np.count_nonzero((b != b[0]).any(axis=0)))


def hgb_ids(keys: np.ndarray):
    """Algorithm 1 stage 1 run sequentially: (group count, gid, gid_loc)."""
    keys = np.ascontiguousarray(keys)
    n = len(keys)
    gid = np.empty(max(n, 1), np.int64)
    loc = np.empty(max(n, 1), np.int64)
    g = lib().oracle_hgb_ids(_key_bytes(keys), _ptr(keys), n, _ptr(gid), _ptr(loc))
    if g < 0:
        raise MemoryError("oracle_hgb_ids")
    return g, gid[:n], loc[:n]


def sort_rows(cols):
    """Rows of a column table sorted lexicographically (first column most
    significant): the canonical form for comparing join outputs as multisets."""
    cols = [np.asarray(c) for c in cols]
    if not cols or len(cols[0]) == 0:
        return cols
    order = np.lexsort(tuple(reversed(cols)))
    return [c[order] for c in cols]
