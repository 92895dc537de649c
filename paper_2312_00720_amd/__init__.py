"""gj: radix-partitioned joins and grouped aggregations on one MI355X.

Thin ctypes binding over libgj.so (C ABI in include/gj.h). It only marshals
arguments: every step of the join and group-by runs in the library's HIP
kernels. torch supplies device memory (through the allocator callback) and the
HIP stream. If libgj.so is missing, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgj.so")

GJ_I32, GJ_I64 = 1, 2
MAT = {"auto": 0, "gftr": 1, "gfur": 2}
JOIN_ALGO = {"auto": 0, "phj": 1, "smj": 2}
GB_ALGO = {"auto": 0, "hash": 1, "sort": 2, "partition": 3, "sort_de": 4}
AGG_OP = {"sum": 1, "count": 2, "min": 3, "max": 4}
DIGIT = {"bits": 0, "hash": 1, "ordered": 2}
ERRORS = {-1: "GJ_EINVAL", -2: "GJ_ENOMEM", -3: "GJ_EHIP", -4: "GJ_EUNSUPPORTED",
          -5: "GJ_ECAPACITY", -6: "GJ_EOVERFLOW"}


class GJError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32)]


class Rel(ctypes.Structure):
    _fields_ = [("key", Col), ("payloads", ctypes.POINTER(Col)), ("n_payloads", ctypes.c_int32),
                ("n_rows", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class RelBatch(ctypes.Structure):
    _fields_ = [("key", Col), ("payloads", ctypes.POINTER(Col)), ("n_payloads", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int64)), ("n_instances", ctypes.c_int32)]


class JoinOpts(ctypes.Structure):
    _fields_ = [("mat", ctypes.c_int32), ("unique_build_keys", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("ht_occupancy", ctypes.c_float),
                ("lds_budget", ctypes.c_int32), ("flags", ctypes.c_uint64), ("algo", ctypes.c_int32),
                ("match_ratio_hint", ctypes.c_float), ("skew_hint", ctypes.c_float)]


class JoinOut(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("r_payloads", ctypes.POINTER(ctypes.c_void_p)),
                ("s_payloads", ctypes.POINTER(ctypes.c_void_p)), ("n_rows", ctypes.c_int64)]


class GbBatch(ctypes.Structure):
    _fields_ = [("key", Col), ("vals", ctypes.POINTER(Col)), ("n_vals", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int64)), ("n_instances", ctypes.c_int32)]


class JoinTuning(ctypes.Structure):
    _fields_ = [("part_log2", ctypes.c_int8 * 32), ("bucket_shift", ctypes.c_int8 * 32),
                ("scatter_variant", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("launches_per_run", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("scratch_bytes", ctypes.c_int64), ("output_bytes", ctypes.c_int64),
                ("unit_capacity", ctypes.c_int64)]


class Agg(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32)]


class GroupByOpts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("mat", ctypes.c_int32), ("radix_bits", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("ht_occupancy", ctypes.c_float),
                ("lds_budget", ctypes.c_int32), ("skew_hint", ctypes.c_float)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class GroupByOut(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("aggs", ctypes.POINTER(ctypes.c_void_p)),
                ("n_groups", ctypes.c_int64)]


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libgj.so; raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2312_00720_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            L.gj_join.restype = ctypes.c_int
            L.gj_join.argtypes = [ctypes.POINTER(Rel), ctypes.POINTER(Rel), ctypes.POINTER(JoinOpts),
                                  ctypes.POINTER(Allocator), vp, ctypes.POINTER(JoinOut)]
            L.gj_join_batch.restype = ctypes.c_int
            L.gj_join_batch.argtypes = [ctypes.POINTER(RelBatch), ctypes.POINTER(RelBatch),
                                        ctypes.POINTER(JoinOpts), ctypes.POINTER(Allocator), vp,
                                        ctypes.POINTER(JoinOut), ctypes.POINTER(ctypes.c_int64)]
            L.gj_partition.restype = ctypes.c_int
            L.gj_partition.argtypes = [Col, ctypes.POINTER(Col), i32, i64, i32, i32, i32, i32,
                                       vp, ctypes.POINTER(vp), vp, vp, ctypes.POINTER(Allocator), vp]
            L.gj_partition_noalloc.restype = ctypes.c_int
            L.gj_partition_noalloc.argtypes = [Col, ctypes.POINTER(Col), i32, i64, i32, i32, i32,
                                               vp, ctypes.POINTER(vp), vp, vp, vp]
            L.gj_partition_noalloc_scratch_bytes.restype = ctypes.c_size_t
            L.gj_partition_noalloc_scratch_bytes.argtypes = []
            L.gj_join_features.restype = ctypes.c_int
            L.gj_join_features.argtypes = [ctypes.POINTER(Rel), ctypes.POINTER(Rel), ctypes.POINTER(JoinOpts),
                                           ctypes.POINTER(ctypes.c_float)]
            L.gj_groupby_features.restype = ctypes.c_int
            L.gj_groupby_features.argtypes = [Col, ctypes.POINTER(Col), i32, ctypes.POINTER(Agg), i32, i64,
                                              ctypes.POINTER(GroupByOpts), ctypes.POINTER(Allocator), vp,
                                              ctypes.POINTER(ctypes.c_float)]
            L.gj_get_cost_constants.restype = ctypes.c_int
            L.gj_get_cost_constants.argtypes = [ctypes.POINTER(ctypes.c_double)] * 3
            L.gj_stream_copy.restype = ctypes.c_int
            L.gj_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
            L.gj_gather_i32.restype = ctypes.c_int
            L.gj_gather_i32.argtypes = [vp, vp, i64, vp, i64, vp]
            L.gj_groupby.restype = ctypes.c_int
            L.gj_groupby.argtypes = [Col, ctypes.POINTER(Col), i32, i64, ctypes.POINTER(Agg), i32,
                                     ctypes.POINTER(GroupByOpts), ctypes.POINTER(Allocator), vp,
                                     ctypes.POINTER(GroupByOut)]
            L.gj_profile_start.restype = ctypes.c_int
            L.gj_profile_start.argtypes = []
            L.gj_profile_stop.restype = ctypes.c_int
            L.gj_profile_stop.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
            fp = ctypes.c_void_p
            L.gj_cost_model.restype = ctypes.c_int
            L.gj_cost_model.argtypes = [ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(ctypes.c_double)]
            L.gj_select.restype = ctypes.c_int
            L.gj_select.argtypes = [ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_float)]
            L.gj_selector_set_weights.restype = ctypes.c_int
            L.gj_selector_set_weights.argtypes = [ctypes.POINTER(ctypes.c_float), i32]
            L.gj_set_cost_constants.restype = ctypes.c_int
            L.gj_set_cost_constants.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
            L.gj_mlp_forward.restype = ctypes.c_int
            L.gj_mlp_forward.argtypes = [fp, fp, fp, i32, fp, ctypes.POINTER(Allocator), vp]
            L.gj_mlp_grad.restype = ctypes.c_int
            L.gj_mlp_grad.argtypes = [fp, fp, fp, fp, i32, fp, fp, ctypes.POINTER(Allocator), vp]
            L.gj_mlp_adam.restype = ctypes.c_int
            L.gj_mlp_adam.argtypes = [fp, fp, fp, fp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, vp]
            pp = ctypes.POINTER(ctypes.c_void_p)
            L.gj_join_plan_create.restype = ctypes.c_int
            L.gj_join_plan_create.argtypes = [ctypes.POINTER(RelBatch), ctypes.POINTER(RelBatch),
                                              ctypes.POINTER(JoinOpts), ctypes.POINTER(JoinTuning), i64,
                                              ctypes.POINTER(Allocator), vp, pp]
            for name in ("gj_plan_run", "gj_plan_launch"):
                getattr(L, name).restype = ctypes.c_int
                getattr(L, name).argtypes = [vp, vp]
            L.gj_plan_capture.restype = ctypes.c_int
            L.gj_plan_capture.argtypes = [vp]
            L.gj_join_plan_result.restype = ctypes.c_int
            L.gj_join_plan_result.argtypes = [vp, vp, ctypes.POINTER(JoinOut), ctypes.POINTER(ctypes.c_int64)]
            L.gj_plan_get_info.restype = ctypes.c_int
            L.gj_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
            L.gj_plan_destroy.restype = ctypes.c_int
            L.gj_plan_destroy.argtypes = [vp]
            L.gj_join_autotune.restype = ctypes.c_int
            L.gj_join_autotune.argtypes = [ctypes.POINTER(RelBatch), ctypes.POINTER(RelBatch),
                                           ctypes.POINTER(JoinOpts), i32, ctypes.POINTER(Allocator), vp,
                                           ctypes.POINTER(JoinTuning)]
            L.gj_groupby_plan_create.restype = ctypes.c_int
            L.gj_groupby_plan_create.argtypes = [ctypes.POINTER(GbBatch), ctypes.POINTER(Agg), i32,
                                                 ctypes.POINTER(GroupByOpts), ctypes.POINTER(Allocator), vp, pp]
            L.gj_groupby_plan_result.restype = ctypes.c_int
            L.gj_groupby_plan_result.argtypes = [vp, vp, ctypes.POINTER(GroupByOut), ctypes.POINTER(ctypes.c_int64)]
            L.gj_groupby_batch.restype = ctypes.c_int
            L.gj_groupby_batch.argtypes = [ctypes.POINTER(GbBatch), ctypes.POINTER(Agg), i32,
                                           ctypes.POINTER(GroupByOpts), ctypes.POINTER(Allocator), vp,
                                           ctypes.POINTER(GroupByOut), ctypes.POINTER(ctypes.c_int64)]
            L.gj_last_error.restype = ctypes.c_char_p
            L.gj_last_error.argtypes = []
            L.gj_version.restype = ctypes.c_char_p
            L.gj_version.argtypes = []
            _lib = L
            _load_shipped_weights(L)
    return _lib


SELECTOR_WEIGHTS = os.path.join(_HERE, "selector_weights.f32")


def _load_shipped_weights(L) -> None:
    """The selector network trained on measured timings ships with the package
    (MLP_PARAMS little-endian float32); once loaded, automatic choices use it
    (else the cost model decides)."""
    if not os.path.exists(SELECTOR_WEIGHTS):
        return
    with open(SELECTOR_WEIGHTS, "rb") as f:
        raw = f.read()
    if len(raw) == 4 * MLP_PARAMS:
        arr = (ctypes.c_float * MLP_PARAMS).from_buffer_copy(raw)
        L.gj_selector_set_weights(arr, MLP_PARAMS)


class _TorchAllocator:
    """Device memory for one library call, from torch's caching allocator on the
    current stream. Blocks handed out as outputs are kept; scratch blocks are
    dropped when the library frees them."""

    def __init__(self, device: torch.device):
        self.device = device
        self.live: dict[int, torch.Tensor] = {}

        def _alloc(nbytes, _ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, _ctx):
            self.live.pop(int(ptr or 0), None)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)
        self.struct = Allocator(self._a, self._f, None)

    def take(self, ptr: int, dtype: torch.dtype, n: int) -> torch.Tensor:
        if n == 0 or not ptr:
            return torch.empty(0, dtype=dtype, device=self.device)
        buf = self.live.pop(int(ptr))
        return buf[: n * torch.empty(0, dtype=dtype).element_size()].view(dtype)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return GJ_I32
    if t.dtype == torch.int64:
        return GJ_I64
    raise TypeError(f"columns must be int32 or int64 tensors, got {t.dtype}")


def _check_cols(cols, n, device):
    for c in cols:
        if c.device != device or not c.is_contiguous() or c.dim() != 1 or c.numel() != n:
            raise ValueError("columns must be contiguous 1-D tensors of equal length on one device")


def _col(t: torch.Tensor) -> Col:
    return Col(t.data_ptr() if t.numel() else None, _dtype_code(t))


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _raise(rc: int):
    if rc != 0:
        raise GJError(rc, lib().gj_last_error().decode())


def join(r_key: torch.Tensor, r_pay, s_key: torch.Tensor, s_pay, *, mat: str = "auto",
         radix_bits: int = 0, passes: int = 0, lds_budget: int = 0, unique_build_keys: bool = False,
         algo: str = "auto", match_ratio_hint: float = 0.0, skew_hint: float = 0.0):
    """Inner equi-join on key. Returns (key, [R payloads], [S payloads]) as
    device tensors; row order is unspecified but deterministic (ascending key
    for algo="smj")."""
    L = lib()
    r_pay, s_pay = list(r_pay), list(s_pay)
    dev = r_key.device
    _check_cols([r_key, *r_pay], r_key.numel(), dev)
    _check_cols([s_key, *s_pay], s_key.numel(), dev)
    rp = (Col * max(1, len(r_pay)))(*[_col(t) for t in r_pay])
    sp = (Col * max(1, len(s_pay)))(*[_col(t) for t in s_pay])
    R = Rel(_col(r_key), rp, len(r_pay), r_key.numel())
    S = Rel(_col(s_key), sp, len(s_pay), s_key.numel())
    o = JoinOpts(MAT[mat], int(unique_build_keys), radix_bits, passes, 0, 0.0, lds_budget, 0, JOIN_ALGO[algo],
                 float(match_ratio_hint), float(skew_hint))
    ro = (ctypes.c_void_p * max(1, len(r_pay)))()
    so = (ctypes.c_void_p * max(1, len(s_pay)))()
    out = JoinOut(None, ro, so, 0)
    A = _TorchAllocator(dev)
    rc = L.gj_join(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o), ctypes.byref(A.struct),
                   _stream(dev), ctypes.byref(out))
    _raise(rc)
    n = out.n_rows
    key = A.take(out.key, r_key.dtype, n)
    rr = [A.take(ro[i], r_pay[i].dtype, n) for i in range(len(r_pay))]
    ss = [A.take(so[i], s_pay[i].dtype, n) for i in range(len(s_pay))]
    return key, rr, ss


def join_batch(r_key: torch.Tensor, r_pay, r_offsets, s_key: torch.Tensor, s_pay, s_offsets, *,
               mat: str = "auto", lds_budget: int = 0):
    """Many independent joins in one call. Columns hold the instances back to back;
    r_offsets / s_offsets (length n+1, host ints) delimit them. Returns
    (key, [R payloads], [S payloads], offsets) with the output concatenated in
    instance order and offsets[i] its first row of instance i."""
    L = lib()
    r_pay, s_pay = list(r_pay), list(s_pay)
    dev = r_key.device
    _check_cols([r_key, *r_pay], r_key.numel(), dev)
    _check_cols([s_key, *s_pay], s_key.numel(), dev)
    n = len(r_offsets) - 1
    if len(s_offsets) != n + 1 or n < 1:
        raise ValueError("offsets of R and S must have the same length >= 2")
    ro = (ctypes.c_int64 * (n + 1))(*[int(x) for x in r_offsets])
    so = (ctypes.c_int64 * (n + 1))(*[int(x) for x in s_offsets])
    rp = (Col * max(1, len(r_pay)))(*[_col(t) for t in r_pay])
    sp = (Col * max(1, len(s_pay)))(*[_col(t) for t in s_pay])
    R = RelBatch(_col(r_key), rp, len(r_pay), ro, n)
    S = RelBatch(_col(s_key), sp, len(s_pay), so, n)
    o = JoinOpts(MAT[mat], 0, 0, 0, 0, 0.0, lds_budget, 0)
    rpo = (ctypes.c_void_p * max(1, len(r_pay)))()
    spo = (ctypes.c_void_p * max(1, len(s_pay)))()
    out = JoinOut(None, rpo, spo, 0)
    offs = (ctypes.c_int64 * (n + 1))()
    A = _TorchAllocator(dev)
    rc = L.gj_join_batch(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o), ctypes.byref(A.struct),
                         _stream(dev), ctypes.byref(out), offs)
    _raise(rc)
    t = out.n_rows
    key = A.take(out.key, r_key.dtype, t)
    rr = [A.take(rpo[i], r_pay[i].dtype, t) for i in range(len(r_pay))]
    ss = [A.take(spo[i], s_pay[i].dtype, t) for i in range(len(s_pay))]
    return key, rr, ss, [int(offs[i]) for i in range(n + 1)]


def _batch_structs(r_key, r_pay, r_offsets, s_key, s_pay, s_offsets):
    r_pay, s_pay = list(r_pay), list(s_pay)
    dev = r_key.device
    _check_cols([r_key, *r_pay], r_key.numel(), dev)
    _check_cols([s_key, *s_pay], s_key.numel(), dev)
    n = len(r_offsets) - 1
    if len(s_offsets) != n + 1 or n < 1:
        raise ValueError("offsets of R and S must have the same length >= 2")
    if int(r_offsets[-1]) != r_key.numel() or int(s_offsets[-1]) != s_key.numel():
        raise ValueError("the last offset must equal the column length")
    keep = dict(ro=(ctypes.c_int64 * (n + 1))(*[int(x) for x in r_offsets]),
                so=(ctypes.c_int64 * (n + 1))(*[int(x) for x in s_offsets]),
                rp=(Col * max(1, len(r_pay)))(*[_col(t) for t in r_pay]),
                sp=(Col * max(1, len(s_pay)))(*[_col(t) for t in s_pay]))
    R = RelBatch(_col(r_key), keep["rp"], len(r_pay), keep["ro"], n)
    S = RelBatch(_col(s_key), keep["sp"], len(s_pay), keep["so"], n)
    return R, S, keep, n


def tuning_table(part_log2=None, bucket_shift=None, scatter_variant: int = 0) -> JoinTuning:
    """A join-plan tuning table; part_log2 / bucket_shift map size class -> value."""
    t = JoinTuning()
    for c, v in (part_log2 or {}).items():
        t.part_log2[int(c)] = int(v)
    for c, v in (bucket_shift or {}).items():
        t.bucket_shift[int(c)] = int(v)
    t.scatter_variant = int(scatter_variant)
    return t


def tuning_dict(t: JoinTuning) -> dict:
    return {"part_log2": {c: int(t.part_log2[c]) for c in range(32) if t.part_log2[c]},
            "bucket_shift": {c: int(t.bucket_shift[c]) for c in range(32) if t.bucket_shift[c]},
            "scatter_variant": int(t.scatter_variant)}


class JoinPlan:
    """A batch of joins planned once and replayed as one HIP graph (gj_join_plan_*).
    The input columns are borrowed: refill them in place and launch again to join
    new data of the same shape. Results are views of the plan's output columns."""

    def __init__(self, r_key, r_pay, r_offsets, s_key, s_pay, s_offsets, *, mat: str = "gftr",
                 lds_budget: int = 0, tuning: JoinTuning | None = None, out_capacity: int = 0):
        L = lib()
        self._p = None
        self.device = r_key.device
        self._inputs = (r_key, list(r_pay), s_key, list(s_pay))
        R, S, self._keep, self.n = _batch_structs(r_key, r_pay, r_offsets, s_key, s_pay, s_offsets)
        self._alloc = _TorchAllocator(self.device)
        o = JoinOpts(MAT[mat], 0, 0, 0, 0, 0.0, lds_budget, 0)
        p = ctypes.c_void_p()
        rc = L.gj_join_plan_create(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o),
                                   ctypes.byref(tuning) if tuning is not None else None, int(out_capacity),
                                   ctypes.byref(self._alloc.struct), _stream(self.device), ctypes.byref(p))
        _raise(rc)
        self._p = p

    def run(self) -> None:
        _raise(lib().gj_plan_run(self._p, _stream(self.device)))

    def capture(self) -> None:
        _raise(lib().gj_plan_capture(self._p))

    def launch(self) -> None:
        _raise(lib().gj_plan_launch(self._p, _stream(self.device)))

    def info(self) -> dict:
        i = PlanInfo()
        _raise(lib().gj_plan_get_info(self._p, ctypes.byref(i)))
        return {k: int(getattr(i, k)) for k, _ in PlanInfo._fields_}

    def result(self):
        """(key, [R payloads], [S payloads], offsets) of the last run; raises
        GJError (GJ_ECAPACITY) with the needed rows when the plan was too small."""
        r_key, r_pay, s_key, s_pay = self._inputs
        ro = (ctypes.c_void_p * max(1, len(r_pay)))()
        so = (ctypes.c_void_p * max(1, len(s_pay)))()
        out = JoinOut(None, ro, so, 0)
        offs = (ctypes.c_int64 * (self.n + 1))()
        rc = lib().gj_join_plan_result(self._p, _stream(self.device), ctypes.byref(out), offs)
        if rc != 0:
            err = GJError(rc, lib().gj_last_error().decode())
            err.n_rows = int(out.n_rows)
            raise err
        t = int(out.n_rows)

        def view(ptr, dtype):
            buf = self._alloc.live[int(ptr)]
            return buf[: t * torch.empty(0, dtype=dtype).element_size()].view(dtype)

        key = view(out.key, r_key.dtype)
        rr = [view(ro[i], r_pay[i].dtype) for i in range(len(r_pay))]
        ss = [view(so[i], s_pay[i].dtype) for i in range(len(s_pay))]
        return key, rr, ss, [int(offs[i]) for i in range(self.n + 1)]

    def close(self) -> None:
        if self._p is not None:
            lib().gj_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GroupByPlan(JoinPlan):
    """Partition group-by of a batch of instances, planned once and replayed as one
    HIP graph (gj_groupby_plan_*). Key and value columns hold the instances back
    to back; offsets (n+1 host ints) delimit them. Inputs are borrowed."""

    def __init__(self, key, vals, offsets, aggs, *, mat: str = "gftr", radix_bits: int = 0):
        L = lib()
        self._p = None
        vals = list(vals)
        self.device = key.device
        _check_cols([key, *vals], key.numel(), self.device)
        self.n = len(offsets) - 1
        if self.n < 1 or int(offsets[-1]) != key.numel():
            raise ValueError("offsets must have >= 2 entries and end at the column length")
        self._inputs = (key, vals)
        self.aggs = [(int(c), op) for c, op in aggs]
        self._keep = dict(off=(ctypes.c_int64 * (self.n + 1))(*[int(x) for x in offsets]),
                          vals=(Col * max(1, len(vals)))(*[_col(t) for t in vals]),
                          aggs=(Agg * max(1, len(aggs)))(*[Agg(int(c), AGG_OP[op]) for c, op in aggs]))
        B = GbBatch(_col(key), self._keep["vals"], len(vals), self._keep["off"], self.n)
        o = GroupByOpts(GB_ALGO["partition"], MAT[mat], radix_bits, 0, 0.0, 0)
        self._alloc = _TorchAllocator(self.device)
        p = ctypes.c_void_p()
        _raise(L.gj_groupby_plan_create(ctypes.byref(B), self._keep["aggs"], len(aggs), ctypes.byref(o),
                                        ctypes.byref(self._alloc.struct), _stream(self.device), ctypes.byref(p)))
        self._p = p

    def result(self):
        """(keys, [aggregate columns], group offsets per instance) of the last run."""
        key, vals = self._inputs
        ao = (ctypes.c_void_p * max(1, len(self.aggs)))()
        out = GroupByOut(None, ao, 0)
        offs = (ctypes.c_int64 * (self.n + 1))()
        _raise(lib().gj_groupby_plan_result(self._p, _stream(self.device), ctypes.byref(out), offs))
        g = int(out.n_groups)

        def view(ptr, dtype):
            buf = self._alloc.live[int(ptr)]
            return buf[: g * torch.empty(0, dtype=dtype).element_size()].view(dtype)

        keys = view(out.key, key.dtype)
        res = [view(ao[i], torch.int64 if op in ("sum", "count") else torch.int32)
               for i, (c, op) in enumerate(self.aggs)]
        return keys, res, [int(offs[i]) for i in range(self.n + 1)]


def join_autotune(r_key, r_pay, r_offsets, s_key, s_pay, s_offsets, *, mat: str = "gftr", lds_budget: int = 0,
                  reps: int = 3) -> JoinTuning:
    """Autotuned plan parameters per size class for this batch (gj_join_autotune)."""
    L = lib()
    R, S, keep, _ = _batch_structs(r_key, r_pay, r_offsets, s_key, s_pay, s_offsets)
    A = _TorchAllocator(r_key.device)
    o = JoinOpts(MAT[mat], 0, 0, 0, 0, 0.0, lds_budget, 0)
    t = JoinTuning()
    _raise(L.gj_join_autotune(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o), int(reps),
                              ctypes.byref(A.struct), _stream(r_key.device), ctypes.byref(t)))
    return t


def partition(key: torch.Tensor, cols=(), *, bit_lo: int = 0, bits: int = 8, passes: int = 0,
              mode: str = "bits", rowid: bool = False):
    """Stable radix partition. Returns (key', [cols'], rowid' or None, offsets[2^bits+1])."""
    L = lib()
    cols = list(cols)
    n = key.numel()
    dev = key.device
    _check_cols([key, *cols], n, dev)
    ok = torch.empty_like(key)
    oc = [torch.empty_like(c) for c in cols]
    orow = torch.empty(n, dtype=torch.int32, device=dev) if rowid else None
    off = torch.empty((1 << bits) + 1, dtype=torch.int32, device=dev)
    ci = (Col * max(1, len(cols)))(*[_col(t) for t in cols])
    co = (ctypes.c_void_p * max(1, len(cols)))(*[t.data_ptr() if n else None for t in oc])
    A = _TorchAllocator(dev)
    rc = L.gj_partition(_col(key), ci, len(cols), n, bit_lo, bits, passes, DIGIT[mode],
                        ok.data_ptr() if n else None, co,
                        orow.data_ptr() if (rowid and n) else None, off.data_ptr(),
                        ctypes.byref(A.struct), _stream(dev))
    _raise(rc)
    return ok, oc, orow, off


def partition_noalloc(key: torch.Tensor, cols, out_key: torch.Tensor, out_cols, out_offsets: torch.Tensor, *,
                      bit_lo: int = 0, bits: int = 8, mode: str = "bits", out_rowid: torch.Tensor | None = None):
    """One-pass stable radix partition into caller-provided outputs, with no
    device allocation by the library (gj_partition_noalloc): out_key and
    out_cols like key and cols, out_offsets int32 of 2^bits + 1, out_rowid
    int32 of n (optional)."""
    L = lib()
    cols, out_cols = list(cols), list(out_cols)
    n = key.numel()
    dev = key.device
    _check_cols([key, *cols, out_key, *out_cols], n, dev)
    if len(out_cols) != len(cols):
        raise ValueError("one output column per input column")
    if out_key.dtype != key.dtype or any(o.dtype != c.dtype for o, c in zip(out_cols, cols)):
        raise ValueError("output columns must have the input columns' dtypes")
    if out_offsets.dtype != torch.int32 or out_offsets.numel() != (1 << bits) + 1:
        raise ValueError("out_offsets must be int32 with 2^bits + 1 entries")
    if out_rowid is not None:
        _check_cols([out_rowid], n, dev)
    ci = (Col * max(1, len(cols)))(*[_col(t) for t in cols])
    co = (ctypes.c_void_p * max(1, len(cols)))(*[t.data_ptr() if n else None for t in out_cols])
    rc = L.gj_partition_noalloc(_col(key), ci, len(cols), n, bit_lo, bits, DIGIT[mode],
                                out_key.data_ptr() if n else None, co,
                                out_rowid.data_ptr() if (out_rowid is not None and n) else None,
                                out_offsets.data_ptr(), _stream(dev))
    _raise(rc)


def groupby(key: torch.Tensor, vals, aggs, *, algo: str = "auto", mat: str = "auto",
            radix_bits: int = 0, lds_budget: int = 0, ht_occupancy: float = 0.0, skew_hint: float = 0.0):
    """Grouped aggregation. `aggs` is a list of (column index, op) with op in
    {"sum", "count", "min", "max"}. Returns (keys, [aggregate columns])."""
    L = lib()
    vals = list(vals)
    n = key.numel()
    dev = key.device
    _check_cols([key, *vals], n, dev)
    vp = (Col * max(1, len(vals)))(*[_col(t) for t in vals])
    ag = (Agg * max(1, len(aggs)))(*[Agg(int(c), AGG_OP[op]) for c, op in aggs])
    o = GroupByOpts(GB_ALGO[algo], MAT[mat], radix_bits, 0, float(ht_occupancy), lds_budget, float(skew_hint))
    ao = (ctypes.c_void_p * max(1, len(aggs)))()
    out = GroupByOut(None, ao, 0)
    A = _TorchAllocator(dev)
    rc = L.gj_groupby(_col(key), vp, len(vals), n, ag, len(aggs), ctypes.byref(o),
                      ctypes.byref(A.struct), _stream(dev), ctypes.byref(out))
    _raise(rc)
    g = out.n_groups
    keys = A.take(out.key, key.dtype, g)
    res = []
    for i, (c, op) in enumerate(aggs):
        dt = torch.int64 if op in ("sum", "count") else vals[c].dtype
        res.append(A.take(ao[i], dt, g))
    return keys, res


def groupby_batch(key: torch.Tensor, vals, offsets, aggs, *, mat: str = "gftr", radix_bits: int = 0):
    """Partition group-by of every instance of a batch in one call (gj_groupby_batch).
    Key and value columns hold the instances back to back; offsets (n+1 host ints)
    delimit them. Returns (keys, [aggregate columns], group offsets per instance)."""
    L = lib()
    vals = list(vals)
    dev = key.device
    _check_cols([key, *vals], key.numel(), dev)
    n = len(offsets) - 1
    if n < 1 or int(offsets[-1]) != key.numel():
        raise ValueError("offsets must have >= 2 entries and end at the column length")
    off = (ctypes.c_int64 * (n + 1))(*[int(x) for x in offsets])
    vp = (Col * max(1, len(vals)))(*[_col(t) for t in vals])
    ag = (Agg * max(1, len(aggs)))(*[Agg(int(c), AGG_OP[op]) for c, op in aggs])
    B = GbBatch(_col(key), vp, len(vals), off, n)
    o = GroupByOpts(GB_ALGO["partition"], MAT[mat], radix_bits, 0, 0.0, 0)
    ao = (ctypes.c_void_p * max(1, len(aggs)))()
    out = GroupByOut(None, ao, 0)
    goff = (ctypes.c_int64 * (n + 1))()
    A = _TorchAllocator(dev)
    _raise(L.gj_groupby_batch(ctypes.byref(B), ag, len(aggs), ctypes.byref(o), ctypes.byref(A.struct),
                              _stream(dev), ctypes.byref(out), goff))
    g = out.n_groups
    keys = A.take(out.key, key.dtype, g)
    res = [A.take(ao[i], torch.int64 if op in ("sum", "count") else vals[c].dtype, g)
           for i, (c, op) in enumerate(aggs)]
    return keys, res, [int(goff[i]) for i in range(n + 1)]


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """dst = src byte for byte with the library's streaming kernel (contiguous
    device tensors of equal byte size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("contiguous tensors of equal byte size")
    _raise(lib().gj_stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream(src.device)))


def gather_i32(map_: torch.Tensor, values: torch.Tensor, out: torch.Tensor) -> None:
    """out[i] = values[map_[i]] (int32 device tensors; out of range map entries give 0)."""
    if map_.dtype != torch.int32 or values.dtype != torch.int32 or out.dtype != torch.int32:
        raise TypeError("int32 tensors")
    if out.numel() != map_.numel():
        raise ValueError("out and map must have equal length")
    _raise(lib().gj_gather_i32(map_.data_ptr(), values.data_ptr(), values.numel(), out.data_ptr(), map_.numel(),
                               _stream(map_.device)))


MLP_PARAMS = 5447
# selector classes (gj.h): partitioned-hash join GFTR / GFUR, hash / sort /
# partition group-by, sort group-by on dictionary-encoded keys, sort-merge join GFTR
CLASSES = ["gftr", "gfur", "hash", "sort", "partition", "sort_de", "smj"]
N_CLASSES = len(CLASSES)
JOIN_CLASSES = (0, 1, 6)
GROUPBY_CLASSES = (2, 3, 4, 5)


def cost_model(features, op_kind: int):
    """Predicted seconds per class (inf for classes invalid for op_kind)."""
    f = (ctypes.c_float * 12)(*[float(x) for x in features])
    out = (ctypes.c_double * N_CLASSES)()
    _raise(lib().gj_cost_model(f, op_kind, out))
    return [out[i] for i in range(N_CLASSES)]


def select(features, op_kind: int):
    """(class index, probabilities) chosen by the network, else the cost model."""
    f = (ctypes.c_float * 12)(*[float(x) for x in features])
    c = ctypes.c_int32(-1)
    p = (ctypes.c_float * N_CLASSES)()
    _raise(lib().gj_select(f, op_kind, ctypes.byref(c), p))
    return c.value, [p[i] for i in range(N_CLASSES)]


def join_features(r_key, r_pay, s_key, s_pay, *, match_ratio_hint: float = 0.0, skew_hint: float = 0.0):
    """The feature vector gj_join's automatic choice uses (host only)."""
    rp = (Col * max(1, len(r_pay)))(*[_col(t) for t in r_pay])
    sp = (Col * max(1, len(s_pay)))(*[_col(t) for t in s_pay])
    R = Rel(_col(r_key), rp, len(r_pay), r_key.numel())
    S = Rel(_col(s_key), sp, len(s_pay), s_key.numel())
    o = JoinOpts(0, 0, 0, 0, 0, 0.0, 0, 0, 0, float(match_ratio_hint), float(skew_hint))
    f = (ctypes.c_float * 12)()
    _raise(lib().gj_join_features(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o), f))
    return [f[i] for i in range(12)]


def groupby_features(key: torch.Tensor, vals, aggs, *, skew_hint: float = 0.0, algo: str = "auto"):
    """The feature vector gj_groupby's automatic choice uses for these columns and
    aggregates (reads the keys once; of the value columns only their widths).
    `algo` picks the sketch kernel gj_groupby would run for that algorithm."""
    vals = list(vals)
    n = key.numel()
    _check_cols([key, *vals], n, key.device)
    vp = (Col * max(1, len(vals)))(*[_col(t) for t in vals])
    ag = (Agg * max(1, len(aggs)))(*[Agg(int(c), AGG_OP[op]) for c, op in aggs])
    o = GroupByOpts(GB_ALGO[algo], 0, 0, 0, 0.0, 0, float(skew_hint))
    f = (ctypes.c_float * 12)()
    A = _TorchAllocator(key.device)
    _raise(lib().gj_groupby_features(_col(key), vp, len(vals), ag, len(aggs), n, ctypes.byref(o),
                                     ctypes.byref(A.struct), _stream(key.device), f))
    return [f[i] for i in range(12)]


def selector_set_weights(params) -> None:
    """Load trained weights (MLP_PARAMS floats) into the library; None unloads them."""
    if params is None:
        _raise(lib().gj_selector_set_weights(None, 0))
        return
    arr = (ctypes.c_float * MLP_PARAMS)(*[float(x) for x in params])
    _raise(lib().gj_selector_set_weights(arr, MLP_PARAMS))


def set_cost_constants(seq_bytes_per_s: float, rand_ratio: float, atomic_rate: float) -> None:
    _raise(lib().gj_set_cost_constants(seq_bytes_per_s, rand_ratio, atomic_rate))


def get_cost_constants() -> tuple:
    """(streaming bytes/s, B_G/B_R, scattered global atomics/s) of the cost model."""
    x = [ctypes.c_double() for _ in range(3)]
    _raise(lib().gj_get_cost_constants(*[ctypes.byref(v) for v in x]))
    return tuple(v.value for v in x)


def mlp_forward(params: torch.Tensor, X: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """Masked softmax probabilities [B, N_CLASSES] of the selector network (FP32, device)."""
    B = X.shape[0]
    out = torch.empty((B, N_CLASSES), dtype=torch.float32, device=X.device)
    A = _TorchAllocator(X.device)
    _raise(lib().gj_mlp_forward(params.data_ptr(), X.data_ptr(), mask.data_ptr(), B, out.data_ptr(),
                                ctypes.byref(A.struct), _stream(X.device)))
    return out


def mlp_grad(params: torch.Tensor, X: torch.Tensor, mask: torch.Tensor, y: torch.Tensor):
    """(loss, gradient) of the batch-mean cross-entropy (FP32, device)."""
    B = X.shape[0]
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    A = _TorchAllocator(X.device)
    _raise(lib().gj_mlp_grad(params.data_ptr(), X.data_ptr(), mask.data_ptr(), y.data_ptr(), B, g.data_ptr(),
                             loss.data_ptr(), ctypes.byref(A.struct), _stream(X.device)))
    return loss, g


def mlp_adam(params, grad, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> None:
    """In-place Adam step on device tensors."""
    _raise(lib().gj_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), t, lr, b1, b2, eps,
                             _stream(params.device)))


def profile_start() -> None:
    """Record HIP events around every later launch of this thread."""
    _raise(lib().gj_profile_start())


def profile_stop() -> dict:
    """Stop recording; returns {kernel: {launches, total_ms, alg_bytes}}."""
    L = lib()
    cap = 128
    buf = (KernelStat * cap)()
    n = ctypes.c_int32(0)
    _raise(L.gj_profile_stop(buf, cap, ctypes.byref(n)))
    return {buf[i].name.decode(): {"launches": int(buf[i].launches), "total_ms": float(buf[i].total_ms),
                                   "alg_bytes": float(buf[i].alg_bytes)}
            for i in range(min(n.value, cap))}


def version() -> str:
    return lib().gj_version().decode()
