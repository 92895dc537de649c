"""GPU parity at the benchmark's full sizes for the workloads that are timed,
beyond the headline join and the g = 2^16 partition group-by.

Large-size protocol (no sorted multiset of 2^28 rows): every output row is
checked by a closed form the oracle can evaluate row by row, and the rest by
order-independent properties that hold at any size.

Joins (|R| = 2^27, |S| = 2^28, 4 + 4 int32 payloads): R keys are a permutation
of 0..|R|-1 (through the bijective splitmix64 widening for 8-byte keys), so an
output row's R payloads must be R.p[inv[key]]; the output holds exactly the
matched S rows, checked by the row count and the oracle's fingerprint of the
multiset of (key, S payloads). The sort-merge join's rows must also come in
ascending key order.

Group-by (N = 2^28, 2 value columns): COUNT, SUM (int64) and MIN/MAX per
present key from direct-address closed forms on the host (integer
index_add / scatter-reduce), for every algorithm and materialization.

Join then group-by (|R| = 2^16, |S| = 2^26): the group-by of the join output
equals the group-by of (R.p[inv[s.key]], s.p) over all S rows.

Batched joins (4096 instances, the autotuned plan): a seeded sample of 64
instances including the largest, each compared with the oracle's join of that
instance alone as a sorted multiset, element by element.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N_R, N_S = 1 << 27, 1 << 28


def _key_values(keys: np.ndarray) -> np.ndarray:
    """The 4-byte value a key was generated from (identity for int32 keys)."""
    from gpu_util import unsplitmix64
    return keys.astype(np.int64) if keys.dtype == np.int32 else unsplitmix64(keys)


C2_CASES = [
    # key bytes, Zipf alpha of the FKs, match ratio, materialization, join algorithm
    (4, 0.0, 1.0, "gfur", "phj"),
    (8, 0.0, 1.0, "gftr", "phj"),
    (4, 1.0, 1.0, "gftr", "phj"),
    (4, 0.0, 0.5, "gftr", "phj"),
    (4, 0.5, 0.5, "gfur", "phj"),
    (8, 1.0, 0.5, "gfur", "phj"),
    (4, 0.0, 1.0, "gftr", "smj"),
    (8, 1.0, 0.5, "gfur", "smj"),
]


@pytest.mark.parametrize("kb,alpha,mr,mat,algo", C2_CASES)
def test_join_full_size_variants(kb, alpha, mr, mat, algo):
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import host, say
    tag = f"full-size join kb={kb} alpha={alpha} mr={mr} {mat} {algo}"
    say(f"{tag}: generating")
    variant = 10 * kb + int(10 * alpha) + (100 if mr < 1 else 0)
    d = dd.pk_fk_join(N_R, N_S, 4, 4, seed=datagen.seed_for(1, variant), alpha=alpha, match_ratio=mr, key_bytes=kb)
    say(f"{tag}: running gj.join")
    k, rp, sp = gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat=mat, algo=algo)
    torch.cuda.synchronize()
    assert k.numel() == d["n_match"]
    say(f"{tag}: R payloads of every row by the closed form")
    rj = _key_values(host(d["r_key"]))
    inv = np.full(N_R, -1, dtype=np.int64)
    inv[rj] = np.arange(N_R, dtype=np.int64)
    del rj
    tk = host(k)
    del k
    if algo == "smj":
        assert np.all(tk[1:] >= tk[:-1]), "sort-merge join emits keys in ascending order"
    tj = _key_values(tk)
    assert tj.min() >= 0 and tj.max() < N_R
    ridx = inv[tj]
    del tj, inv
    for j in range(4):
        np.testing.assert_array_equal(host(rp[j]), host(d["r_pay"][j])[ridx])
    del ridx, rp
    say(f"{tag}: fingerprint of (key, S payloads) against the matched S rows")
    got = oracle.rows_fingerprint([tk] + [host(x) for x in sp])
    del sp
    sk = host(d["s_key"])
    sj = _key_values(sk)
    matched = (sj >= 0) & (sj < N_R)
    assert int(matched.sum()) == d["n_match"]
    want = oracle.rows_fingerprint([sk[matched]] + [host(x)[matched] for x in d["s_pay"]])
    assert got == want


def _expected_groups(k: np.ndarray, vals):
    """COUNT, SUM, MIN, MAX per present key of {0..g-1}, in key order, from
    int64 index_add and scatter_reduce on the host."""
    import torch
    kt = torch.from_numpy(k.astype(np.int64))
    g = int(kt.max()) + 1
    cnt = torch.zeros(g, dtype=torch.int64).index_add_(0, kt, torch.ones_like(kt))
    present = torch.nonzero(cnt).flatten()
    out = {"key": present.numpy(), "count": cnt[present].numpy(), "sum": [], "min": [], "max": []}
    for v in vals:
        vt = torch.from_numpy(v.astype(np.int64))
        out["sum"].append(torch.zeros(g, dtype=torch.int64).index_add_(0, kt, vt)[present].numpy())
        out["min"].append(torch.full((g,), 2**31 - 1, dtype=torch.int64)
                          .scatter_reduce(0, kt, vt, "amin")[present].numpy())
        out["max"].append(torch.full((g,), -2**31, dtype=torch.int64)
                          .scatter_reduce(0, kt, vt, "amax")[present].numpy())
    return out


GB_AGGS = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]


def _check_groups(keys, res, want, what):
    from gpu_util import host
    gk = host(keys).astype(np.int64)
    order = np.argsort(gk, kind="stable")
    np.testing.assert_array_equal(gk[order], want["key"], err_msg=what)
    np.testing.assert_array_equal(host(res[0])[order], want["count"], err_msg=what)
    for c, (si, mi, xi) in enumerate([(1, 2, 3), (4, 5, 6)]):
        np.testing.assert_array_equal(host(res[si])[order], want["sum"][c], err_msg=what)
        np.testing.assert_array_equal(host(res[mi])[order], want["min"][c], err_msg=what)
        np.testing.assert_array_equal(host(res[xi])[order], want["max"][c], err_msg=what)


GB_ALGOS = [("hash", "auto"), ("sort", "gftr"), ("sort", "gfur"), ("partition", "gftr"), ("partition", "gfur"),
            ("sort_de", "gftr")]


@pytest.mark.parametrize("log2g,alpha", [(4, 0.0), (16, 0.0), (26, 0.0), (16, 1.0)])
def test_groupby_full_size_grid(log2g, alpha):
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import host, say
    n, g = 1 << 28, 1 << log2g
    say(f"full-size group-by g=2^{log2g} alpha={alpha}: generating")
    d = dd.groupby_input(n, g, 2, seed=datagen.seed_for(2, 200 + log2g + (50 if alpha else 0)), alpha=alpha)
    say("closed forms on the host")
    want = _expected_groups(host(d["key"]), [host(v) for v in d["vals"]])
    for algo, mat in GB_ALGOS:
        say(f"full-size group-by g=2^{log2g} alpha={alpha}: {algo} {mat}")
        keys, res = gj.groupby(d["key"], d["vals"], GB_AGGS, algo=algo, mat=mat)
        torch.cuda.synchronize()
        _check_groups(keys, res, want, f"{algo}/{mat}")
        if algo.startswith("sort"):
            gk = host(keys)
            assert np.all(gk[1:] > gk[:-1]), "sort group-by emits ascending keys"
        del keys, res


def test_join_then_groupby_full_size():
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import host, say
    n_r, n_s = 1 << 16, 1 << 26
    say("pipeline |R|=2^16 |S|=2^26: generating (the benchmark's inputs)")
    d = dd.pk_fk_join(n_r, n_s, 1, 1, seed=datagen.seed_for(2, 900))
    aggs = [(0, "count"), (0, "sum"), (0, "min"), (0, "max")]
    k, rp, sp = gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat="auto")
    gk, res = gj.groupby(rp[0], [sp[0]], aggs, algo="auto")
    torch.cuda.synchronize()
    say("pipeline: closed form on the host")
    rk = host(d["r_key"]).astype(np.int64)
    inv = np.empty(n_r, np.int64)
    inv[rk] = np.arange(n_r)
    gkey = host(d["r_pay"][0])[inv[host(d["s_key"]).astype(np.int64)]]
    uk, idx = np.unique(gkey, return_inverse=True)
    it = torch.from_numpy(idx.astype(np.int64))
    vt = torch.from_numpy(host(d["s_pay"][0]).astype(np.int64))
    m = len(uk)
    cnt = torch.zeros(m, dtype=torch.int64).index_add_(0, it, torch.ones_like(it)).numpy()
    sm = torch.zeros(m, dtype=torch.int64).index_add_(0, it, vt).numpy()
    mn = torch.full((m,), 2**31 - 1, dtype=torch.int64).scatter_reduce(0, it, vt, "amin").numpy()
    mx = torch.full((m,), -2**31, dtype=torch.int64).scatter_reduce(0, it, vt, "amax").numpy()
    got = host(gk)
    order = np.argsort(got, kind="stable")
    np.testing.assert_array_equal(got[order], uk)
    np.testing.assert_array_equal(host(res[0])[order], cnt)
    np.testing.assert_array_equal(host(res[1])[order], sm)
    np.testing.assert_array_equal(host(res[2])[order], mn)
    np.testing.assert_array_equal(host(res[3])[order], mx)


def test_join_batch_plan_per_instance():
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import canon, host, say
    n = 4096
    r_sz, s_sz = datagen.batch_sizes(n, datagen.seed_for(3, n))
    say(f"batch of {n} joins: generating (the benchmark's inputs)")
    d = dd.join_batch(r_sz, s_sz, 2, datagen.seed_for(3, n + 1))
    cols = (d["r_key"], d["r_pay"], d["r_off"], d["s_key"], d["s_pay"], d["s_off"])
    say("batch: autotuning and capturing the plan")
    tuning = gj.join_autotune(*cols, mat="gftr", reps=1)
    plan = gj.JoinPlan(*cols, mat="gftr", tuning=tuning)
    plan.capture()
    plan.launch()
    plan.launch()  # a replay over the same inputs
    key, rp, sp, off = plan.result()
    torch.cuda.synchronize()
    assert off[-1] == int(s_sz.sum())
    g = datagen.rng(3131)
    sample = set(g.choice(n, size=63, replace=False).tolist()) | {int(np.argmax(s_sz))}
    r_off, s_off = d["r_off"], d["s_off"]
    for i in sorted(sample):
        ro, so = slice(r_off[i], r_off[i + 1]), slice(s_off[i], s_off[i + 1])
        t = slice(off[i], off[i + 1])
        got = [host(key[t])] + [host(x[t]) for x in rp] + [host(x[t]) for x in sp]
        want = oracle.join(host(d["r_key"][ro]), [host(x[ro]) for x in d["r_pay"]],
                           host(d["s_key"][so]), [host(x[so]) for x in d["s_pay"]])
        assert len(got[0]) == len(want[0]) == s_sz[i], i
        for a, b in zip(canon(got), canon(want)):
            np.testing.assert_array_equal(a, b, err_msg=f"instance {i}")
    plan.close()
