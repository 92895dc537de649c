"""Failure handling forced from the host: an allocator that returns NULL at its
k-th request makes every entry point fail with GJ_ENOMEM, and each block the
library obtained before that is handed back, so no output stays allocated.
Kernels already enqueued only touch blocks that are released in stream order,
and every kernel exits normally."""
import ctypes

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

GJ_ENOMEM = -2


class FailingAllocator:
    """torch-backed device memory that fails at request number `fail_at`
    (1-based; 0 = never) and tracks live blocks."""

    def __init__(self, gj, fail_at: int):
        import torch
        self.live, self.requests, self.fail_at = {}, 0, fail_at

        def _alloc(nbytes, _ctx):
            self.requests += 1
            if self.requests == self.fail_at:
                return None
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, _ctx):
            self.live.pop(int(ptr or 0))

        self._a, self._f = gj._ALLOC_FN(_alloc), gj._FREE_FN(_free)
        self.struct = gj.Allocator(self._a, self._f, None)


def _sweep(gj, call, what):
    """Runs call(alloc) once to count requests, then fails each request in turn."""
    import torch
    from gpu_util import say
    ok = FailingAllocator(gj, 0)
    assert call(ok) == 0, gj.lib().gj_last_error()
    total = ok.requests
    assert total > 0
    say(f"{what}: {total} allocation requests; failing each in turn")
    for k in sorted(set(np.linspace(1, total, min(total, 24)).astype(int).tolist())):
        a = FailingAllocator(gj, k)
        rc = call(a)
        torch.cuda.synchronize()
        assert rc == GJ_ENOMEM, (what, k, rc, gj.lib().gj_last_error())
        assert not a.live, (what, k, len(a.live))


def test_enomem_releases_everything():
    import paper_2312_00720_amd as gj
    from gpu_util import dev
    L = gj.lib()
    d = datagen.pk_fk_join(5000, 20000, 2, 1, seed=datagen.seed_for(0, 31), match_ratio=0.8)
    rk, sk = dev(d["r_key"]), dev(d["s_key"])
    rp, sp = [dev(x) for x in d["r_pay"]], [dev(x) for x in d["s_pay"]]
    R = gj.Rel(gj._col(rk), (gj.Col * 2)(*[gj._col(t) for t in rp]), 2, rk.numel())
    S = gj.Rel(gj._col(sk), (gj.Col * 1)(*[gj._col(t) for t in sp]), 1, sk.numel())
    for mat in (1, 2):
        def join(a, mat=mat):
            ro, so = (ctypes.c_void_p * 2)(), (ctypes.c_void_p * 1)()
            out = gj.JoinOut(None, ro, so, 0)
            o = gj.JoinOpts(mat, 0, 0, 0, 0, 0.0, 0, 0)
            rc = L.gj_join(ctypes.byref(R), ctypes.byref(S), ctypes.byref(o), ctypes.byref(a.struct),
                           gj._stream(rk.device), ctypes.byref(out))
            if rc != 0:
                assert out.key is None and out.n_rows == 0
            return rc
        _sweep(gj, join, f"join mat={mat}")

    g = datagen.groupby_input(30000, 700, 2, seed=datagen.seed_for(2, 31))
    key, vals = dev(g["key"]), [dev(v) for v in g["vals"]]
    vp = (gj.Col * 2)(*[gj._col(t) for t in vals])
    aggs = (gj.Agg * 3)(gj.Agg(0, 2), gj.Agg(0, 1), gj.Agg(1, 4))
    for algo in (1, 2, 3):
        def groupby(a, algo=algo):
            ao = (ctypes.c_void_p * 3)()
            out = gj.GroupByOut(None, ao, 0)
            o = gj.GroupByOpts(algo, 1, 0, 0, 0.0, 0)
            rc = L.gj_groupby(gj._col(key), vp, 2, key.numel(), aggs, 3, ctypes.byref(o), ctypes.byref(a.struct),
                              gj._stream(key.device), ctypes.byref(out))
            if rc != 0:
                assert out.key is None and out.n_groups == 0
            return rc
        _sweep(gj, groupby, f"group-by algo={algo}")

    import torch
    ok_ = torch.empty_like(key)

    def partition(a):
        return L.gj_partition(gj._col(key), None, 0, key.numel(), 0, 12, 2, 0, ok_.data_ptr(), None, None, None,
                              ctypes.byref(a.struct), gj._stream(key.device))
    _sweep(gj, partition, "partition")
