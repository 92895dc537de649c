"""Host-side error paths of the C ABI, forced from the host with no device
work: more than 2^31 - 1 rows in a relation returns GJ_EOVERFLOW before any
device memory is touched (row identifiers are 32-bit), and argument errors
return GJ_EINVAL. The pointers passed are never dereferenced on these paths."""
import ctypes

import pytest

GJ_EINVAL, GJ_EOVERFLOW = -1, -6
FAKE = 0x1000  # a non-null placeholder; every call here fails before using it
BIG = 1 << 31


@pytest.fixture(scope="module")
def gj():
    import paper_2312_00720_amd as gj
    gj.lib()
    return gj


def _join(gj, n_r, n_s):
    L = gj.lib()
    R = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, n_r)
    S = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, n_s)
    out = gj.JoinOut(None, None, None, 0)
    return L.gj_join(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out)), out


def test_join_overflow(gj):
    for n_r, n_s in ((BIG, 10), (10, BIG), (BIG + 5, BIG)):
        rc, out = _join(gj, n_r, n_s)
        assert rc == GJ_EOVERFLOW, gj.lib().gj_last_error()
        assert out.key is None and out.n_rows == 0
        assert b"2^31-1" in gj.lib().gj_last_error()


def test_join_limit_is_accepted_by_the_checks(gj):
    # 2^31 - 1 rows pass the row check; a null key column is then the error
    L = gj.lib()
    R = gj.Rel(gj.Col(None, gj.GJ_I32), None, 0, BIG - 1)
    S = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, 1)
    out = gj.JoinOut(None, None, None, 0)
    assert L.gj_join(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out)) == GJ_EINVAL
    assert b"null data" in L.gj_last_error()


def test_groupby_and_partition_overflow(gj):
    L = gj.lib()
    aggs = (gj.Agg * 1)(gj.Agg(0, gj.AGG_OP["count"]))
    ao = (ctypes.c_void_p * 1)()
    out = gj.GroupByOut(None, ao, 0)
    rc = L.gj_groupby(gj.Col(FAKE, gj.GJ_I32), None, 0, BIG, aggs, 1, None, None, None, ctypes.byref(out))
    assert rc == GJ_EOVERFLOW and out.n_groups == 0
    rc = L.gj_partition(gj.Col(FAKE, gj.GJ_I32), None, 0, BIG, 0, 8, 1, 0, FAKE, None, None, None, None, None)
    assert rc == GJ_EOVERFLOW
    rc = L.gj_partition_noalloc(gj.Col(FAKE, gj.GJ_I32), None, 0, BIG, 0, 8, 0, FAKE, None, None, FAKE, None)
    assert rc == GJ_EOVERFLOW


def test_join_batch_overflow(gj):
    L = gj.lib()
    off_r = (ctypes.c_int64 * 3)(0, BIG // 2, BIG)
    off_s = (ctypes.c_int64 * 3)(0, 5, 10)
    R = gj.RelBatch(gj.Col(FAKE, gj.GJ_I32), None, 0, off_r, 2)
    S = gj.RelBatch(gj.Col(FAKE, gj.GJ_I32), None, 0, off_s, 2)
    out = gj.JoinOut(None, None, None, 0)
    offs = (ctypes.c_int64 * 3)()
    rc = L.gj_join_batch(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out), offs)
    assert rc == GJ_EOVERFLOW


def test_argument_errors(gj):
    L = gj.lib()
    # key dtypes differ
    R = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, 10)
    S = gj.Rel(gj.Col(FAKE, gj.GJ_I64), None, 0, 10)
    out = gj.JoinOut(None, None, None, 0)
    assert L.gj_join(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out)) == GJ_EINVAL
    # negative rows, unknown dtype
    R = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, -1)
    S = gj.Rel(gj.Col(FAKE, gj.GJ_I32), None, 0, 10)
    assert L.gj_join(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out)) == GJ_EINVAL
    R = gj.Rel(gj.Col(FAKE, 7), None, 0, 10)
    assert L.gj_join(ctypes.byref(R), ctypes.byref(S), None, None, None, ctypes.byref(out)) == GJ_EINVAL
    # the no-allocation partition takes one pass only, and needs the offsets
    assert L.gj_partition_noalloc(gj.Col(FAKE, gj.GJ_I32), None, 0, 10, 0, 9, 0, FAKE, None, None, FAKE,
                                  None) == GJ_EINVAL
    assert L.gj_partition_noalloc(gj.Col(FAKE, gj.GJ_I32), None, 0, 10, 0, 8, 0, FAKE, None, None, None,
                                  None) == GJ_EINVAL
    assert L.gj_partition_noalloc_scratch_bytes() == 8 << 20
