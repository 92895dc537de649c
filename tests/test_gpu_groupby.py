"""GPU parity: hash-, sort- and partition-based group-by (Sections 4.2, 4.1.3,
4.3) against the oracle. Integer aggregates are compared exactly, groups
matched by key."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

AGGS = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]


def gpu_groupby(keys, vals, aggs, **kw):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    say(f"groupby n={len(keys)} key={keys.dtype} nv={len(vals)} {kw}")
    k, res = gj.groupby(dev(keys), [dev(v) for v in vals], aggs, **kw)
    return host(k), [host(r) for r in res]


def expected(keys, vals, aggs):
    o = oracle.groupby(keys, vals)
    cols = []
    for c, op in aggs:
        if op == "count":
            cols.append(o["count"])
        else:
            cols.append(o[op][c])
    return o["key"], cols


def check(keys, vals, aggs=AGGS, sorted_out=False, **kw):
    gk, gcols = gpu_groupby(keys, vals, aggs, **kw)
    ek, ecols = expected(keys, vals, aggs)
    assert len(gk) == len(ek)
    if sorted_out:
        np.testing.assert_array_equal(gk, ek)  # sort-based group-by emits keys in order
    order = np.argsort(gk, kind="stable")
    np.testing.assert_array_equal(gk[order], ek)
    for (c, op), g, e in zip(aggs, gcols, ecols):
        assert g.dtype == (np.int64 if op in ("sum", "count") else np.asarray(vals[c]).dtype)
        np.testing.assert_array_equal(g[order], e, err_msg=f"{op}({c})")
    return gk, gcols


ALGOS = [("partition", "gftr"), ("partition", "gfur"), ("hash", "auto"), ("sort", "gftr"), ("sort", "gfur"),
         ("sort_de", "gftr")]


@pytest.mark.parametrize("algo,mat", ALGOS)
@pytest.mark.parametrize("n,card,alpha", [(1000, 7, 0.0), (200003, 16, 0.0), (200003, 3000, 0.0),
                                          (200003, 150000, 0.0), (300001, 4096, 1.0)])
def test_groupby_matches_oracle(algo, mat, n, card, alpha):
    d = datagen.groupby_input(n, card, 2, seed=datagen.seed_for(2, card + n), alpha=alpha)
    check(d["key"], d["vals"], algo=algo, mat=mat, sorted_out=algo.startswith("sort"))


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("g_card,alpha", [(1, 0.0), (200, 0.0), (70000, 0.0), (5000, 1.1)])
def test_sort_de_sparse_keys(kb, g_card, alpha):
    """Dictionary-encoded sort group-by (Section 4.4) on sparse keys: g distinct
    values spread over the whole key range (all 4 or 8 key bytes vary, so the
    plain sort needs 4 or 8 passes, the codes ceil(log2 g / 8)); keys come out
    in ascending signed order, including negative keys and both extremes."""
    g = datagen.rng(900 + g_card + kb)
    lo, hi = (-2**31, 2**31 - 1) if kb == 4 else (-2**63, 2**63 - 1)
    dom = np.unique(g.integers(lo, hi, size=g_card, endpoint=True, dtype=np.int64))
    if g_card > 1:
        dom[0], dom[-1] = lo, hi
    ranks = datagen.zipf_ranks(g, 250007, len(dom), alpha) - 1
    keys = dom[g.permutation(len(dom))][ranks].astype(np.int32 if kb == 4 else np.int64)
    vals = [g.integers(-2**31, 2**31, size=len(keys)).astype(np.int32) for _ in range(2)]
    check(keys, vals, algo="sort_de", sorted_out=True)
    check(keys, vals, AGGS[:4], algo="sort_de", sorted_out=True)
    check(keys, [], [(0, "count")], algo="sort_de", sorted_out=True)


@pytest.mark.parametrize("kb,nv", [(4, 1), (4, 2), (8, 2)])
def test_partition_many_groups_per_partition(kb, nv):
    """About 1200 groups in each of 256 partitions: the aggregation's table and
    records take over 53 KB of LDS, fewer than three 256-thread workgroups'
    worth, which selects its 1024-thread workgroups."""
    d = datagen.groupby_input(600001, 300000, nv, seed=30 + kb + nv, key_bytes=kb)
    aggs = AGGS if nv == 2 else AGGS[:4]
    check(d["key"], d["vals"], aggs, algo="partition", mat="gftr", radix_bits=8)
    check(d["key"], d["vals"], aggs, algo="partition", mat="gfur", radix_bits=8)


@pytest.mark.parametrize("algo", ["partition", "hash", "sort"])
def test_groupby_int64_keys(algo):
    d = datagen.groupby_input(100000, 5000, 2, seed=12, key_bytes=8)
    check(d["key"], d["vals"], algo=algo, sorted_out=(algo == "sort"))


@pytest.mark.parametrize("algo", ["partition", "hash", "sort"])
def test_groupby_edge_keys(algo):
    """Keys at the extremes of the signed range, including the value the LDS
    tables use as their empty marker, and a single group."""
    g = datagen.rng(3)
    for dt, lo, hi in [(np.int32, -2**31, 2**31 - 1), (np.int64, -2**63, 2**63 - 1)]:
        keys = np.array([lo, hi, 0, -1, lo, lo, 5, hi] * 1000, dtype=dt)
        vals = [g.integers(-2**20, 2**20 + 1, size=len(keys)).astype(np.int32) for _ in range(2)]
        check(keys, vals, algo=algo, sorted_out=(algo == "sort"))
    keys = np.full(50000, 42, np.int32)
    vals = [g.integers(-2**20, 2**20 + 1, size=50000).astype(np.int32) for _ in range(2)]
    check(keys, vals, algo=algo, sorted_out=(algo == "sort"))


@pytest.mark.parametrize("algo", ["partition", "hash", "sort"])
def test_groupby_tiny_and_empty(algo):
    for n in (0, 1, 2, 17):
        keys = np.arange(n, dtype=np.int32) % 3
        vals = [np.arange(n, dtype=np.int32) - 5, np.full(n, 7, np.int32)]
        check(keys, vals, algo=algo, sorted_out=(algo == "sort"))


def test_aggregate_list_variants():
    d = datagen.groupby_input(50000, 300, 3, seed=4)
    for aggs in ([(0, "count")], [(2, "max"), (0, "sum"), (2, "max"), (1, "min")], [(1, "sum")] * 3):
        for algo in ("partition", "hash", "sort"):
            check(d["key"], d["vals"], aggs=aggs, algo=algo)


def test_partition_overflow_falls_back():
    """Two partitions for 20000 distinct keys overflow the per-partition LDS table;
    the result must still be exact."""
    d = datagen.groupby_input(60000, 20000, 2, seed=5)
    check(d["key"], d["vals"], algo="partition", radix_bits=1)


@pytest.mark.parametrize("kb", [4, 8])
def test_partition_skewed_keys(kb):
    """Zipf 1.0 keys: the hottest key's partition holds several times the mean
    partition's work units, which switches MIN/MAX to reading the record before
    the atomic. Results stay exact."""
    d = datagen.groupby_input(2_000_000, 20000, 2, seed=41, alpha=1.0, key_bytes=kb)
    check(d["key"], d["vals"], algo="partition", mat="gftr")
    check(d["key"], d["vals"], algo="partition", mat="gfur")


def test_partition_slice_overflow_falls_back():
    """Partitions of 150000 rows are discovered in slices of 65536 rows, and each
    slice here holds about 14000 distinct keys, more than a slice's LDS table: the
    partition group-by hands over to hash group-by and the result stays exact
    (the merge must not read the counts the overflowing slices never produced)."""
    d = datagen.groupby_input(300000, 30000, 2, seed=31)
    check(d["key"], d["vals"], algo="partition", radix_bits=1)
    check(d["key"], d["vals"], algo="partition", radix_bits=1, mat="gfur")


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_hash_partial_lds_records(alpha):
    """More groups than LDS records: the first group ids keep LDS records, the
    rest aggregate with global atomics (uniform and skewed keys)."""
    d = datagen.groupby_input(200000, 3000, 2, seed=66, alpha=alpha)
    check(d["key"], d["vals"], algo="hash", lds_budget=4000)


def test_hash_ids_follow_the_first_rows():
    """Group ids go to the keys of the first rows (inserted by one workgroup
    before the full grid), which under skew are the frequent keys; when not every
    group fits in LDS, those lowest ids keep LDS records. HGB emits groups in id
    order, so those keys come first in its output. Here the first 2048 rows hold
    1014 distinct keys, and 1638 is what a 64 KB budget holds of 40-byte records
    (7 aggregates)."""
    d = datagen.groupby_input(400000, 20000, 2, seed=5, alpha=1.0)
    gk, _ = check(d["key"], d["vals"], algo="hash")
    first = np.unique(d["key"][:2048])
    assert len(first) == 1014 and len(gk) == 19167
    assert np.isin(first, gk[:1638]).all()


@pytest.mark.parametrize("occ", [0.0, 0.9, 8.0])
def test_hash_table_sizing(occ):
    """The global table is sized from the group-count estimate at load `occ`; at
    8.0 it is far too small, rows run out of probes, and the insert runs again
    on a table of 1.5 slots per row. Results are exact either way."""
    d = datagen.groupby_input(300000, 50000, 2, seed=67)
    check(d["key"], d["vals"], algo="hash", ht_occupancy=occ)
    d = datagen.groupby_input(100000, 7, 2, seed=68, key_bytes=8)
    check(d["key"], d["vals"], algo="hash", ht_occupancy=occ)


@pytest.mark.parametrize("g_card,budget,alpha", [(3000, 8192, 0.0), (2000, 16384, 1.0), (20000, 0, 0.0),
                                                  (65000, 0, 1.0), (5, 0, 0.0), (200000, 0, 0.0),
                                                  (10000, 8192, 0.5)])
def test_hash_sliced_lds_records(g_card, budget, alpha):
    """Every group in LDS, the ids cut into up to 64 consecutive ranges that each
    fit one workgroup's LDS (budget 0: 160 KB); each (row chunk, id range)
    workgroup aggregates its chunk's rows of that range, several ranges reading
    the rows' resolved group ids."""
    d = datagen.groupby_input(300001, g_card, 2, seed=69 + g_card, alpha=alpha)
    check(d["key"], d["vals"], algo="hash", lds_budget=budget)
    d = datagen.groupby_input(100003, g_card, 2, seed=70 + g_card, alpha=alpha, key_bytes=8)
    check(d["key"], d["vals"], algo="hash", lds_budget=budget)


@pytest.mark.parametrize("nv,alpha", [(4, 0.0), (8, 0.0), (4, 1.0)])
def test_hash_sliced_many_value_columns(nv, alpha):
    """Sliced hash aggregation with 4 and 8 value columns: queued rows carry
    their row index (their values are read when the queue is drained) rather than
    the values themselves, and the records take 16 aggregates."""
    d = datagen.groupby_input(250007, 20000, nv, seed=90 + nv, alpha=alpha)
    aggs = [(0, "count")] + [(c, "sum") for c in range(nv)] + [(c, "min") for c in range(nv)][:14 - nv]
    aggs += [(nv - 1, "max")]
    check(d["key"], d["vals"], aggs, algo="hash")
    check(d["key"], d["vals"], aggs, algo="hash", lds_budget=24576)


@pytest.mark.parametrize("g_card", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nv,v64", [(1, False), (2, False), (4, False), (2, True), (8, True)])
def test_hash_few_groups(g_card, nv, v64):
    """A handful of groups (register accumulators per thread, folded once per
    wave): every column type and count, int32 extremes in the values, a ragged
    row count, and the automatic choice on the same input."""
    n = 300007
    d = datagen.groupby_input(n, g_card, nv, seed=datagen.seed_for(11, g_card * 10 + nv))
    vals = d["vals"]
    if v64:
        g = datagen.rng(400 + g_card + nv)
        vals = [g.integers(-2**62, 2**62, size=n, dtype=np.int64) for _ in range(nv)]
        vals[0][:2] = [np.iinfo(np.int64).min, np.iinfo(np.int64).max]
    else:
        vals[0][:2] = [np.iinfo(np.int32).min, np.iinfo(np.int32).max]
    aggs = [(0, "count")] + [(c, op) for c in range(nv) for op in ("sum", "min", "max")][:15]
    check(d["key"], vals, aggs, algo="hash")
    check(d["key"], vals, aggs, algo="auto")


@pytest.mark.parametrize("card", [3000, 20])
def test_hash_misaligned_keys(card):
    """Keys one element past a 16-byte boundary: the hash insert's cached kernel
    (16-byte runs) steps aside for the row-by-row one, with the same result."""
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    d = datagen.groupby_input(100003, card, 2, seed=datagen.seed_for(13, card))
    keys, vals = d["key"], d["vals"]
    kd = dev(np.concatenate([keys[:1], keys]))[1:]
    vd = [dev(np.concatenate([v[:1], v]))[1:] for v in vals]
    assert kd.data_ptr() % 16 != 0
    say(f"groupby misaligned keys card={card}")
    gk, res = gj.groupby(kd, vd, AGGS, algo="hash")
    gk = host(gk)
    ek, ecols = expected(keys, vals, AGGS)
    order = np.argsort(gk, kind="stable")
    np.testing.assert_array_equal(gk[order], ek)
    for r, e in zip(res, ecols):
        np.testing.assert_array_equal(host(r)[order], e)


@pytest.mark.parametrize("algo", ["hash", "sort_de"])
def test_eight_byte_keys_cached_insert(algo):
    """8-byte keys with few groups go through the insert's LDS cache of resolved
    keys, whose empty marker is a key value (-2^63 + 1): rows holding that key
    bypass the cache. Keys at and around the marker and both extremes."""
    g = datagen.rng(77)
    dom = np.array([-2**63, -2**63 + 1, -2**63 + 2, -1, 0, 1, 2**63 - 1], np.int64)
    dom = np.concatenate([dom, g.integers(-2**62, 2**62, size=300, dtype=np.int64)])
    keys = dom[g.integers(0, len(dom), size=200003)]
    vals = [g.integers(-2**31, 2**31, size=len(keys)).astype(np.int32) for _ in range(2)]
    check(keys, vals, algo=algo, sorted_out=(algo == "sort_de"))


def test_hash_global_aggregation_path():
    d = datagen.groupby_input(100000, 2000, 2, seed=6)
    check(d["key"], d["vals"], algo="hash", lds_budget=64)


@pytest.mark.parametrize("bits", [1, 4, 9, 16])
def test_partition_bits_do_not_change_results(bits):
    d = datagen.groupby_input(120000, 1500, 2, seed=7, alpha=0.8)
    check(d["key"], d["vals"], algo="partition", radix_bits=bits)


@pytest.mark.parametrize("algo", ["partition", "sort"])
def test_groupby_deterministic(algo):
    d = datagen.groupby_input(150000, 20000, 2, seed=8)
    a = gpu_groupby(d["key"], d["vals"], AGGS, algo=algo)
    b = gpu_groupby(d["key"], d["vals"], AGGS, algo=algo)
    np.testing.assert_array_equal(a[0], b[0])
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_partition_oversized_partitions(dt):
    """Partitions above one discovery slice (65536 rows) are discovered by several
    workgroups and merged: few groups, a Zipf-hot key, and the key value that the
    LDS tables use as their empty marker inside an oversized partition."""
    g = datagen.rng(21)
    n = 400000
    lo = np.iinfo(dt).min
    keys = np.where(g.uniform(size=n) < 0.7, 0, g.integers(-3, 4, size=n)).astype(dt)
    keys[g.choice(n, 5000, replace=False)] = lo
    vals = [g.integers(-2**20, 2**20 + 1, size=n).astype(np.int32) for _ in range(2)]
    check(keys, vals, algo="partition")
    check(keys, vals, algo="partition", radix_bits=2, mat="gfur")
    d = datagen.groupby_input(n, 16, 2, seed=22, alpha=1.0)
    check(d["key"], d["vals"], algo="partition")


@pytest.mark.parametrize("algo,mat", ALGOS)
@pytest.mark.parametrize("kb,card,alpha", [(4, 3000, 0.0), (8, 150000, 0.0), (4, 4096, 1.1), (8, 5, 0.0)])
def test_eight_byte_values(algo, mat, kb, card, alpha):
    """8-byte value columns (Section 5.2's 8-byte payloads), alone and next to a
    4-byte column: SUM in int64 (wrapping like two's complement once values reach
    2^62), MIN and MAX as int64, the 4-byte column's MIN and MAX as int32."""
    d = datagen.groupby_input(200003, card, 1, seed=datagen.seed_for(2, 300 + card), alpha=alpha, key_bytes=kb)
    g = datagen.rng(301 + card)
    v8 = g.integers(-2**62, 2**62, size=len(d["key"]), dtype=np.int64)
    v8[:3] = [np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0]
    gk, gcols = check(d["key"], [d["vals"][0], v8], algo=algo, mat=mat, sorted_out=algo.startswith("sort"))
    assert gcols[2].dtype == np.int32 and gcols[5].dtype == np.int64
    check(d["key"], [v8], AGGS[:4], algo=algo, mat=mat)


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("n,card,alpha", [(1, 1, 0.0), (1000, 7, 0.0), (200003, 3000, 0.0),
                                          (1 << 20, 1 << 16, 0.0), ((1 << 21) + 77, 1 << 20, 0.0),
                                          (300001, 4096, 1.0)])
@pytest.mark.parametrize("algo", ["auto", "hash"])
def test_group_count_sketch_matches_oracle(kb, n, card, alpha, algo):
    """The group-count estimate an automatic choice feeds the selector equals the
    oracle's HyperLogLog estimate, through both sketch kernels (with the
    partition histogram for automatic choices, without it for the hash
    group-by's table sizing), and the varying key bytes match."""
    import paper_2312_00720_amd as gj
    from gpu_util import dev, say
    d = datagen.groupby_input(n, card, 0, seed=datagen.seed_for(7, card + n), alpha=alpha)
    keys = d["key"] if kb == 4 else datagen.widen_keys(d["key"])
    say(f"sketch n={n} card={card} kb={kb} algo={algo}")
    vals = [dev(np.zeros(n, np.int32))]
    aggs = [(0, "count"), (0, "sum"), (0, "max")]  # a 4-word record: 16 bytes per group
    f = gj.groupby_features(dev(keys), vals, aggs, algo=algo)
    # keys one element past a 16-byte boundary take the row-by-row loads
    shifted = dev(np.concatenate([keys[:1], keys]))[1:]
    assert shifted.data_ptr() % 16 != 0
    assert gj.groupby_features(shifted, vals, aggs, algo=algo) == f
    est = max(1.0, oracle.hll_estimate(keys))
    # one float ulp: a register off by one moves this feature by far more
    want = np.float32(np.log2(est) / 32.0)
    assert abs(np.float32(f[3]) - want) <= np.spacing(want), (f[3], want)
    want = np.float32(np.log2(est * 16.0) / 32.0)  # the records' LDS bytes
    assert abs(np.float32(f[10]) - want) <= np.spacing(want), (f[10], want)
    assert f[5] == np.float32(1 / 8)
    assert f[6] == np.float32((oracle.varying_key_bytes(keys) or kb) / 8.0)
