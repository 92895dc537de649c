"""Pins for the group-by, partition and hash-group-ID oracles.

Group-by: one group key, reducible aggregates (Section 2.2). Partition: the
radix-partition primitive of Section 2.3. Group IDs: Algorithm 1, stage 1
(Section 4.2).
"""
import numpy as np
import pytest

import datagen
import oracle


def brute_groupby(keys, vals):
    groups = {}
    for i, k in enumerate(keys):
        groups.setdefault(int(k), []).append(i)
    out = []
    for k in sorted(groups):
        rows = groups[k]
        rec = [k, len(rows)]
        for v in vals:
            xs = [int(v[i]) for i in rows]
            rec += [sum(xs), min(xs), max(xs)]
        out.append(tuple(rec))
    return out


def flatten(res, nv):
    out = []
    for gi in range(len(res["key"])):
        rec = [int(res["key"][gi]), int(res["count"][gi])]
        for v in range(nv):
            rec += [int(res["sum"][v][gi]), int(res["min"][v][gi]), int(res["max"][v][gi])]
        out.append(tuple(rec))
    return out


@pytest.mark.parametrize("n,lo,hi,nv,dt", [
    (0, 0, 3, 2, np.int32), (1, 4, 4, 1, np.int32), (300, 0, 9, 2, np.int32),
    (300, -20, 20, 3, np.int32), (200, -2**31, -2**31 + 2, 1, np.int32),
    (200, 2**31 - 3, 2**31 - 1, 2, np.int32), (250, -7, 7, 2, np.int64),
    (100, -2**63, -2**63 + 3, 1, np.int64),
])
def test_groupby_matches_brute_force(n, lo, hi, nv, dt):
    g = datagen.rng(n + nv)
    keys = g.integers(lo, hi, size=n, endpoint=True, dtype=np.int64).astype(dt)
    vals = [g.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32) for _ in range(nv)]
    assert flatten(oracle.groupby(keys, vals), nv) == brute_groupby(keys, vals)


@pytest.mark.parametrize("card,alpha", [(16, 0.0), (4096, 0.0), (4096, 1.0), (1 << 16, 0.0)])
def test_groupby_direct_address_closed_form(card, alpha):
    d = datagen.groupby_input(1 << 17, card, 2, seed=datagen.seed_for(2, card), alpha=alpha)
    k = d["key"].astype(np.int64)
    res = oracle.groupby(d["key"], d["vals"])
    present = np.nonzero(np.bincount(k, minlength=card))[0]
    np.testing.assert_array_equal(res["key"], present)
    np.testing.assert_array_equal(res["count"], np.bincount(k, minlength=card)[present])
    for v in range(2):
        x = d["vals"][v].astype(np.int64)
        s = np.zeros(card, np.int64)
        np.add.at(s, k, x)
        mn = np.full(card, 2**31 - 1, np.int64)
        np.minimum.at(mn, k, x)
        mx = np.full(card, -2**31, np.int64)
        np.maximum.at(mx, k, x)
        np.testing.assert_array_equal(res["sum"][v], s[present])
        np.testing.assert_array_equal(res["min"][v], mn[present])
        np.testing.assert_array_equal(res["max"][v], mx[present])
    # invariants: counts sum to N, sums add up, MIN <= MAX, one group per distinct key
    assert res["count"].sum() == len(k)
    assert res["sum"][0].sum() == d["vals"][0].astype(np.int64).sum()
    assert np.all(res["min"][1] <= res["max"][1])
    assert len(res["key"]) == len(np.unique(k))


def test_groupby_value_range_is_closed():
    d = datagen.groupby_input(1 << 16, 4, 1, seed=1, lo=-2, hi=2)
    assert d["vals"][0].min() == -2 and d["vals"][0].max() == 2


def _digit_py(key, key_bytes, mode, lo, bits):
    return (oracle.digit_source(int(key), key_bytes, mode) >> lo) & ((1 << bits) - 1)


def test_hash_digit_matches_published_vectors():
    # MurmurHash3_x86_32 of the empty input reduces to the finalizer of the seed;
    # its published values for seeds 1 and 0xffffffff pin the finalizer.
    assert oracle.digit_source(1, 4, oracle.DIGIT_HASH) == 0x514E28B7
    assert oracle.digit_source(-1, 4, oracle.DIGIT_HASH) == 0x81F16F39
    assert oracle.digit_source(0, 4, oracle.DIGIT_HASH) == 0
    # 8-byte keys hash the xor of their two words
    assert oracle.digit_source(1 << 32, 8, oracle.DIGIT_HASH) == 0x514E28B7
    # ordered digits flip the sign bit, so unsigned order equals signed order
    assert oracle.digit_source(-2**31, 4, oracle.DIGIT_ORDERED) == 0
    assert oracle.digit_source(2**31 - 1, 4, oracle.DIGIT_ORDERED) == 2**32 - 1
    assert oracle.digit_source(-1, 8, oracle.DIGIT_ORDERED) == 2**63 - 1
    assert oracle.digit_source(-5, 4, oracle.DIGIT_BITS) == 2**32 - 5


@pytest.mark.parametrize("mode", [oracle.DIGIT_BITS, oracle.DIGIT_HASH, oracle.DIGIT_ORDERED])
@pytest.mark.parametrize("key_bytes,lo,bits", [(4, 0, 3), (4, 5, 4), (4, 28, 4), (8, 0, 5), (8, 40, 6)])
def test_partition_is_stable_sort_by_digit(mode, key_bytes, lo, bits):
    keys = datagen.raw_keys(500, seed=lo + bits + mode, key_bytes=key_bytes)
    perm, hist = oracle.partition(keys, lo, bits, mode)
    dig = [_digit_py(k, key_bytes, mode, lo, bits) for k in keys]
    want = sorted(range(len(keys)), key=lambda i: dig[i])  # Python's sort is stable
    assert list(perm) == want
    assert list(hist) == [dig.count(d) for d in range(1 << bits)]


def test_partition_invariants_large():
    keys = datagen.raw_keys(1 << 18, seed=4)
    perm, hist = oracle.partition(keys, 3, 8, oracle.DIGIT_BITS)
    assert np.array_equal(np.sort(perm), np.arange(len(keys)))
    d = (keys.view(np.uint32).astype(np.int64) >> 3) & 255
    ds = d[perm]
    assert np.all(np.diff(ds) >= 0)
    same = np.diff(ds) == 0
    assert np.all(np.diff(perm)[same] > 0)
    np.testing.assert_array_equal(hist, np.bincount(d, minlength=256))


@pytest.mark.parametrize("n,card", [(0, 1), (1, 1), (200, 7), (500, 500), (1000, 3)])
def test_hgb_ids(n, card):
    g = datagen.rng(n * 3 + card)
    keys = g.integers(0, card, size=n, dtype=np.int64).astype(np.int32)
    ng, gid, loc = oracle.hgb_ids(keys)
    first = {}
    want_gid, want_loc = [], []
    for i, k in enumerate(keys):
        k = int(k)
        if k not in first:
            first[k] = (i, len(first))
            want_gid.append(first[k][1])
        else:
            want_gid.append(-1)
        want_loc.append(first[k][0])
    assert ng == len(first)
    assert list(gid) == want_gid and list(loc) == want_loc
    # bijection of inserting rows onto 0..g-1; locations share the key
    ids = gid[gid >= 0]
    assert sorted(ids.tolist()) == list(range(ng))
    assert np.all(keys[loc] == keys)


def brute_groupby64(keys, vals):
    """Per distinct key: count, and per column the sum reduced to a signed 64-bit
    value (two's complement), min and max, with Python integers."""
    out = []
    for rec in brute_groupby(keys, vals):
        rec = list(rec)
        for v in range(len(vals)):
            s = rec[2 + 3 * v] % 2**64
            rec[2 + 3 * v] = s - 2**64 if s >= 2**63 else s
        out.append(tuple(rec))
    return out


@pytest.mark.parametrize("n,nv,span", [(0, 1, 10), (1, 2, 10), (400, 2, 2**62), (300, 3, 2**40),
                                       (200, 1, 2**63)])
def test_groupby64_matches_brute_force(n, nv, span):
    """8-byte value columns (oracle_groupby64): brute force per key; with values
    up to 2^63 in magnitude the sums wrap, as 64-bit two's complement does."""
    g = datagen.rng(7000 + n + nv)
    keys = g.integers(-5, 6, size=n).astype(np.int32)
    vals = [g.integers(-span, span, size=n, dtype=np.int64) for _ in range(nv)]
    if n > 3:
        vals[0][:2] = [np.iinfo(np.int64).min, np.iinfo(np.int64).max]
    assert flatten(oracle.groupby(keys, vals), nv) == brute_groupby64(keys, vals)


def test_groupby64_closed_form_and_mixed_widths():
    """A 4-byte and an 8-byte column together: np.add.at / np.minimum.at /
    np.maximum.at on int64 per key of {0..g-1}; the 4-byte column's results equal
    the int32 oracle's."""
    d = datagen.groupby_input(1 << 15, 777, 1, seed=91)
    g = datagen.rng(92)
    v8 = g.integers(-2**50, 2**50, size=1 << 15, dtype=np.int64)
    res = oracle.groupby(d["key"], [d["vals"][0], v8])
    k = d["key"].astype(np.int64)
    present = np.nonzero(np.bincount(k, minlength=777))[0]
    np.testing.assert_array_equal(res["key"], present)
    s = np.zeros(777, np.int64)
    np.add.at(s, k, v8)
    mn = np.full(777, np.iinfo(np.int64).max)
    np.minimum.at(mn, k, v8)
    mx = np.full(777, np.iinfo(np.int64).min)
    np.maximum.at(mx, k, v8)
    np.testing.assert_array_equal(res["sum"][1], s[present])
    np.testing.assert_array_equal(res["min"][1], mn[present])
    np.testing.assert_array_equal(res["max"][1], mx[present])
    r32 = oracle.groupby(d["key"], d["vals"])
    for f in ("sum", "min", "max"):
        np.testing.assert_array_equal(res[f][0], r32[f][0])
