"""Pins for the join oracle: brute force, closed forms and invariants.

The join is the inner equi-join of Section 2.2; R holds primary keys and S
foreign keys in the paper's workloads (Section 5.1.1), and the many-to-many
case is covered in Section 5.1 (many-to-many joins).
"""
import numpy as np
import pytest

import datagen
import oracle


def brute_join(r_key, r_pay, s_key, s_pay):
    """Nested loops in plain Python: for s in S, for r in R, emit on equal keys."""
    rows = []
    for j in range(len(s_key)):
        for i in range(len(r_key)):
            if int(r_key[i]) == int(s_key[j]):
                rows.append((int(s_key[j]),) + tuple(int(p[i]) for p in r_pay)
                            + tuple(int(p[j]) for p in s_pay))
    return rows


def as_rows(cols):
    return list(zip(*[[int(x) for x in c] for c in cols])) if cols and len(cols[0]) else []


CASES = [
    # (n_r, n_s, key range lo, hi, c_r, c_s, dtype)
    (0, 0, 0, 3, 1, 1, np.int32),
    (0, 17, 0, 3, 1, 2, np.int32),
    (13, 0, 0, 3, 2, 1, np.int32),
    (1, 1, 5, 5, 1, 1, np.int32),
    (40, 60, 0, 7, 2, 2, np.int32),           # many duplicates on both sides
    (64, 200, -5, 5, 1, 3, np.int32),         # negative keys
    (100, 100, 0, 1000, 3, 1, np.int32),      # sparse matches
    (30, 50, -2**31, -2**31 + 3, 1, 1, np.int32),   # INT32_MIN neighbourhood
    (30, 50, 2**31 - 4, 2**31 - 1, 1, 1, np.int32),  # INT32_MAX neighbourhood
    (50, 80, -3, 3, 2, 2, np.int64),
    (50, 80, 2**63 - 3, 2**63 - 1, 1, 1, np.int64),
]


@pytest.mark.parametrize("case", CASES)
def test_join_matches_nested_loops(case):
    n_r, n_s, lo, hi, c_r, c_s, dt = case
    g = datagen.rng(7 + n_r + n_s)
    r_key = g.integers(lo, hi, size=n_r, endpoint=True, dtype=np.int64).astype(dt)
    s_key = g.integers(lo, hi, size=n_s, endpoint=True, dtype=np.int64).astype(dt)
    r_pay = datagen.payload_columns(g, n_r, c_r)
    s_pay = datagen.payload_columns(g, n_s, c_s)
    got = as_rows(oracle.join(r_key, r_pay, s_key, s_pay))
    want = brute_join(r_key, r_pay, s_key, s_pay)
    assert got == want  # same rows in the same (S order, then R order) sequence


def test_join_count_is_sum_over_keys():
    d = datagen.many_to_many_join(3000, 4000, 500, 1, 1, seed=11)
    ir, js = oracle.join_pairs(d["r_key"], d["s_key"])
    ku, cr = np.unique(d["r_key"], return_counts=True)
    ks, cs = np.unique(d["s_key"], return_counts=True)
    common, ia, ib = np.intersect1d(ku, ks, return_indices=True)
    assert len(ir) == int(np.sum(cr[ia].astype(np.int64) * cs[ib]))
    assert np.all(d["r_key"][ir] == d["s_key"][js])


@pytest.mark.parametrize("key_bytes", [4, 8])
@pytest.mark.parametrize("mr,alpha", [(1.0, 0.0), (0.5, 0.0), (1.0, 1.0), (0.25, 0.5)])
def test_pkfk_closed_form(key_bytes, mr, alpha):
    n_r, n_s = 1 << 12, 1 << 14
    d = datagen.pk_fk_join(n_r, n_s, 2, 2, seed=datagen.seed_for(1, 3), alpha=alpha,
                           match_ratio=mr, key_bytes=key_bytes)
    cols = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    # |T| is exactly round(mr * |S|) for a PK-FK join (each S row has <= 1 partner).
    assert len(cols[0]) == int(round(mr * n_s)) == d["n_match"]
    # Direct-address closed form: R.key is a bijection from rows onto its key
    # set, so every matched S row s yields (s.key, R.p[inv[s.key]], s.p).
    pos = {int(k): i for i, k in enumerate(d["r_key"])}
    match = np.array([int(k) in pos for k in d["s_key"]])
    j = np.nonzero(match)[0]
    i = np.array([pos[int(k)] for k in d["s_key"][j]], dtype=np.int64)
    want = [d["s_key"][j]] + [p[i] for p in d["r_pay"]] + [p[j] for p in d["s_pay"]]
    for a, b in zip(cols, want):
        np.testing.assert_array_equal(a, b)


def test_rows_fingerprint_matches_python():
    g = datagen.rng(3)
    cols = [g.integers(-50, 50, size=37).astype(np.int32),
            g.integers(-2**40, 2**40, size=37).astype(np.int64)]
    M = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    s1 = s2 = 0
    for i in range(37):
        h = 0x243F6A8885A308D3
        for c in cols:
            h = mix(h ^ (int(c[i]) & M))
        s1 = (s1 + h) & M
        s2 = (s2 + h * h) & M
    assert oracle.rows_fingerprint(cols) == (37, s1, s2)


@pytest.mark.parametrize("key_bytes", [4, 8])
def test_join_fingerprint_matches_materialized(key_bytes):
    d = datagen.many_to_many_join(2000, 3000, 700, 2, 3, seed=5, key_bytes=key_bytes)
    cols = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    assert oracle.join_fingerprint(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"]) \
        == oracle.rows_fingerprint(cols)


def test_fingerprint_detects_a_changed_row():
    d = datagen.pk_fk_join(256, 1024, 1, 1, seed=9)
    cols = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    fp = oracle.rows_fingerprint(cols)
    cols[1] = cols[1].copy()
    cols[1][17] ^= 1
    assert oracle.rows_fingerprint(cols) != fp
    # and is blind to row order, as intended
    perm = np.random.default_rng(0).permutation(len(cols[0]))
    cols2 = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    assert oracle.rows_fingerprint([c[perm] for c in cols2]) == fp


def test_sort_rows_canonical():
    a = [np.array([2, 1, 2, 1]), np.array([0, 5, -1, 5]), np.array([9, 8, 7, 6])]
    s = oracle.sort_rows(a)
    assert as_rows(s) == sorted(as_rows(a))
