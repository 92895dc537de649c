"""GPU parity for batch plans (graph-captured persistent runs): each instance's
output equals the oracle's join of that instance alone; a plan's run equals the
eager batch call row for row; graph replays, refilled inputs, several instance
groups, capacity errors and tuning tables never change a result."""
import os

import numpy as np
import pytest

import datagen
import oracle
from test_gpu_batch import make_batch

pytestmark = pytest.mark.gpu


def uneven_sizes(n, seed, lo=0, hi=14):
    g = datagen.rng(seed)
    sizes = []
    for _ in range(n):
        nr = int(round(2 ** g.uniform(lo, hi)))
        sizes.append((nr, nr * int(g.integers(4, 17))))
    return sizes


def device_batch(b):
    from gpu_util import dev
    return (dev(b["r_key"]), [dev(x) for x in b["r_pay"]], list(b["r_off"]),
            dev(b["s_key"]), [dev(x) for x in b["s_pay"]], list(b["s_off"]))


def host_cols(res):
    from gpu_util import host
    k, rp, sp, off = res
    return [host(k)] + [host(x) for x in rp] + [host(x) for x in sp], off


def check_vs_oracle(parts, cols, off):
    from gpu_util import canon
    assert off[0] == 0 and off[-1] == len(cols[0])
    for i, p in enumerate(parts):
        want = oracle.join(p["r_key"], p["r_pay"], p["s_key"], p["s_pay"])
        got = [c[off[i]:off[i + 1]] for c in cols]
        assert len(got[0]) == len(want[0]), i
        for a, e in zip(canon(got), canon(want)):
            np.testing.assert_array_equal(a, e)


def run_plan(plan, mode):
    if mode == "eager":
        plan.run()
    else:
        plan.capture()
        plan.launch()
    return host_cols(plan.result())


@pytest.mark.parametrize("mat", ["gftr", "gfur"])
@pytest.mark.parametrize("mode", ["eager", "graph"])
def test_plan_matches_oracle_and_eager_batch(mat, mode):
    import paper_2312_00720_amd as gj
    from gpu_util import say
    sizes = uneven_sizes(80, 31)
    sizes[3] = (0, 50)
    sizes[9] = (40, 0)
    sizes[10] = (1, 1)
    parts, b = make_batch(sizes, seed=5000)
    d = device_batch(b)
    say(f"plan {mat} {mode}: {len(parts)} instances")
    plan = gj.JoinPlan(*d, mat=mat)
    cols, off = run_plan(plan, mode)
    check_vs_oracle(parts, cols, off)
    # same kernels and parameters as the eager batch call: identical rows in identical order
    ecols, eoff = host_cols(gj.join_batch(*d, mat=mat))
    assert off == eoff
    for a, e in zip(cols, ecols):
        np.testing.assert_array_equal(a, e)
    info = plan.info()
    assert info["groups"] == 1 and info["launches_per_run"] > 0
    plan.close()


def test_graph_replays_and_refilled_inputs():
    """Replays interleaved with other device work give the eager result each time;
    refilling the borrowed inputs in place joins the new data."""
    import torch
    import paper_2312_00720_amd as gj
    from gpu_util import dev, say
    sizes = uneven_sizes(50, 32, hi=13)
    parts, b = make_batch(sizes, seed=6000)
    d = device_batch(b)
    plan = gj.JoinPlan(*d, mat="gftr")
    plan.capture()
    ecols, eoff = host_cols(gj.join_batch(*d, mat="gftr"))
    for rep in range(3):
        say(f"replay {rep}")
        junk = torch.arange(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        plan.launch()
        cols, off = host_cols(plan.result())
        assert off == eoff and int(junk) > 0
        for a, e in zip(cols, ecols):
            np.testing.assert_array_equal(a, e)
    # new data of the same shape, written into the same device buffers
    parts2, b2 = make_batch(sizes, seed=7000)
    d[0].copy_(dev(b2["r_key"]))
    d[3].copy_(dev(b2["s_key"]))
    for j in range(2):
        d[1][j].copy_(dev(b2["r_pay"][j]))
        d[4][j].copy_(dev(b2["s_pay"][j]))
    plan.launch()
    cols, off = host_cols(plan.result())
    check_vs_oracle(parts2, cols, off)
    plan.close()


def test_plan_several_groups_int64_many_to_many(monkeypatch):
    import paper_2312_00720_amd as gj
    monkeypatch.setenv("GJ_PLAN_GROUP_ROWS", "20000")
    g = datagen.rng(33)
    sizes = [(int(g.integers(1, 3000)), int(g.integers(1, 5000))) for _ in range(30)]
    for key_bytes, many, mat in [(4, True, "gftr"), (8, False, "gfur"), (8, True, "gftr")]:
        parts, b = make_batch(sizes, seed=8000 + key_bytes, key_bytes=key_bytes, many=many)
        d = device_batch(b)
        cap = sum(len(oracle.join(p["r_key"], p["r_pay"], p["s_key"], p["s_pay"])[0]) for p in parts)
        plan = gj.JoinPlan(*d, mat=mat, out_capacity=max(cap, 1))
        assert plan.info()["groups"] > 1
        cols, off = run_plan(plan, "graph")
        check_vs_oracle(parts, cols, off)
        plan.close()


def test_plan_capacity_error_reports_needed_rows():
    import paper_2312_00720_amd as gj
    g = datagen.rng(34)
    sizes = [(int(g.integers(1, 2000)), int(g.integers(1, 4000))) for _ in range(10)]
    parts, b = make_batch(sizes, seed=9000, many=True)
    need = sum(len(oracle.join(p["r_key"], p["r_pay"], p["s_key"], p["s_pay"])[0]) for p in parts)
    assert need > 10
    d = device_batch(b)
    plan = gj.JoinPlan(*d, mat="gftr", out_capacity=need // 2)
    plan.capture()
    plan.launch()
    with pytest.raises(gj.GJError) as ei:
        plan.result()
    assert ei.value.n_rows == need
    plan.close()


def test_tuning_tables_never_change_results():
    import paper_2312_00720_amd as gj
    sizes = uneven_sizes(40, 35, lo=6, hi=15)
    parts, b = make_batch(sizes, seed=9500)
    d = device_batch(b)
    rng = datagen.rng(36)
    for trial in range(3):
        t = gj.tuning_table({c: int(rng.integers(6, 13)) for c in range(16)},
                            {c: int(rng.integers(0, 2)) for c in range(16)}, int(rng.integers(0, 15)))
        plan = gj.JoinPlan(*d, mat="gftr" if trial % 2 == 0 else "gfur", tuning=t)
        cols, off = run_plan(plan, "graph")
        check_vs_oracle(parts, cols, off)
        plan.close()


@pytest.mark.parametrize("variant", list(range(1, 15)))
def test_every_scatter_shape_matches_oracle(variant):
    """Each compiled scatter shape (variant 14 is the wide 16384-row tile) gives
    the oracle's join on uneven instances, 8-byte keys included."""
    import paper_2312_00720_amd as gj
    sizes = uneven_sizes(12, 38 + variant, lo=0, hi=15)
    parts, b = make_batch(sizes, seed=9600 + variant, key_bytes=8 if variant % 2 else 4)
    d = device_batch(b)
    plan = gj.JoinPlan(*d, mat="gftr" if variant % 3 else "gfur", tuning=gj.tuning_table(scatter_variant=variant))
    cols, off = run_plan(plan, "eager")
    check_vs_oracle(parts, cols, off)
    plan.close()


def test_autotune_gives_a_valid_table():
    import paper_2312_00720_amd as gj
    sizes = uneven_sizes(40, 37, lo=8, hi=14)
    parts, b = make_batch(sizes, seed=9700)
    d = device_batch(b)
    t = gj.join_autotune(*d, mat="gftr", reps=2)
    td = gj.tuning_dict(t)
    classes = {int(np.floor(np.log2(r))) for r, s in sizes if r > 0 and s > 0}
    assert set(td["part_log2"]) == classes
    assert all(9 <= v <= 12 for v in td["part_log2"].values())
    assert 0 <= td["scatter_variant"] <= 14
    plan = gj.JoinPlan(*d, mat="gftr", tuning=t)
    cols, off = run_plan(plan, "graph")
    check_vs_oracle(parts, cols, off)
    plan.close()


# ---- group-by batches ----------------------------------------------------------

GB_AGGS = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]


def gb_batch(sizes, seed, key_bytes=4, alpha=0.0):
    parts = []
    for i, (n, card) in enumerate(sizes):
        parts.append(datagen.groupby_input(n, max(1, card), 2, seed=seed + i, alpha=alpha, key_bytes=key_bytes))
    kd = np.int32 if key_bytes == 4 else np.int64
    key = np.concatenate([p["key"] for p in parts]) if parts else np.zeros(0, kd)
    vals = [np.concatenate([p["vals"][c] for p in parts]).astype(np.int32) for c in range(2)]
    off = np.concatenate([[0], np.cumsum([len(p["key"]) for p in parts])])
    return parts, key, vals, [int(x) for x in off]


def check_gb(parts, res):
    from gpu_util import host
    keys, cols, off = res
    keys = host(keys)
    cols = [host(c) for c in cols]
    assert off[0] == 0 and off[-1] == len(keys)
    for i, p in enumerate(parts):
        o = oracle.groupby(p["key"], p["vals"])
        k = keys[off[i]:off[i + 1]]
        order = np.argsort(k, kind="stable")
        np.testing.assert_array_equal(k[order], o["key"])
        for (c, op), col in zip(GB_AGGS, cols):
            want = o["count"] if op == "count" else o[op][c]
            np.testing.assert_array_equal(col[off[i]:off[i + 1]][order], want, err_msg=f"instance {i} {op}({c})")


@pytest.mark.parametrize("mat", ["gftr", "gfur"])
def test_groupby_plan_matches_oracle(mat):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, say
    g = datagen.rng(41)
    sizes = []
    for _ in range(60):
        n = int(round(2 ** g.uniform(0, 16)))
        sizes.append((n, int(round(2 ** g.uniform(0, max(0.0, np.log2(max(n, 1))))))))
    sizes[4] = (0, 1)
    sizes[8] = (1, 1)
    parts, key, vals, off = gb_batch(sizes, seed=12000)
    say(f"group-by plan {mat}: {len(parts)} instances, {len(key)} rows")
    plan = gj.GroupByPlan(dev(key), [dev(v) for v in vals], off, GB_AGGS, mat=mat)
    plan.run()
    check_gb(parts, plan.result())
    plan.capture()
    for _ in range(2):
        plan.launch()
        check_gb(parts, plan.result())
    plan.close()


@pytest.mark.parametrize("kb,mat", [(4, "gftr"), (8, "gfur")])
def test_groupby_batch_eager_matches_plan_and_oracle(kb, mat):
    """gj_groupby_batch: one call returns caller-owned columns of exactly the
    group count, equal row for row to the plan's result, and the oracle's
    aggregates per instance (empty and one-row instances included)."""
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    g = datagen.rng(43 + kb)
    sizes = [(int(round(2 ** g.uniform(0, 15))), int(g.integers(1, 3000))) for _ in range(40)]
    sizes[5] = (0, 1)
    sizes[6] = (1, 1)
    parts, key, vals, off = gb_batch(sizes, seed=15000 + kb, key_bytes=kb)
    say(f"group-by batch {kb}-byte keys {mat}: {len(parts)} instances, {len(key)} rows")
    keys, cols, goff = gj.groupby_batch(dev(key), [dev(v) for v in vals], off, GB_AGGS, mat=mat)
    assert len(goff) == len(parts) + 1 and goff[-1] == keys.numel()
    assert all(c.numel() == keys.numel() for c in cols)
    check_gb(parts, (keys, cols, goff))
    plan = gj.GroupByPlan(dev(key), [dev(v) for v in vals], off, GB_AGGS, mat=mat)
    plan.run()
    pk, pc, poff = plan.result()
    assert poff == goff
    np.testing.assert_array_equal(host(pk), host(keys))
    for a, b in zip(pc, cols):
        np.testing.assert_array_equal(host(a), host(b))
    plan.close()


def test_groupby_plan_groups_skew_int64(monkeypatch):
    import paper_2312_00720_amd as gj
    from gpu_util import dev
    monkeypatch.setenv("GJ_PLAN_GROUP_ROWS", "50000")
    g = datagen.rng(42)
    sizes = [(int(g.integers(1, 40000)), int(g.integers(1, 3000))) for _ in range(25)]
    for key_bytes, alpha in [(4, 1.0), (8, 0.0)]:
        parts, key, vals, off = gb_batch(sizes, seed=13000 + key_bytes, key_bytes=key_bytes, alpha=alpha)
        plan = gj.GroupByPlan(dev(key), [dev(v) for v in vals], off, GB_AGGS)
        assert plan.info()["groups"] > 1
        plan.capture()
        plan.launch()
        check_gb(parts, plan.result())
        plan.close()


def test_groupby_plan_large_partitions_and_single_groups():
    """Instances whose partitions exceed one discovery slice (few keys), one-group
    instances, and radix_bits forcing large partitions."""
    import paper_2312_00720_amd as gj
    from gpu_util import dev
    sizes = [(300000, 3), (200000, 1), (5000, 5000), (70000, 1)]
    parts, key, vals, off = gb_batch(sizes, seed=14000)
    for bits in (0, 1):
        plan = gj.GroupByPlan(dev(key), [dev(v) for v in vals], off, GB_AGGS, radix_bits=bits)
        plan.capture()
        plan.launch()
        check_gb(parts, plan.result())
        plan.close()
