"""GPU parity of grouped aggregation at the ends of the int32 value range
(Section 2.2 aggregates; SUM and COUNT in int64, MIN and MAX in int32).

Values sit at or next to INT32_MIN and INT32_MAX, so that a group's SUM passes
2^31 in both directions within a few rows (a 32-bit accumulator anywhere would
wrap), a group of only INT32_MAX values has MIN = INT32_MAX and one of only
INT32_MIN values has MAX = INT32_MIN (the values the MIN and MAX records start
from), and single-row groups hold one extreme. Uniform keys and Zipf-skewed
keys (which take the partition group-by's skew path for MIN and MAX) run
through every algorithm, both materializations, and the batched plan, against
the oracle's exact int64 group-by."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1


def extreme_input(n: int, g_card: int, alpha: float, seed: int):
    g = datagen.rng(seed)
    keys = (datagen.zipf_ranks(g, n, g_card, alpha) - 1).astype(np.int32)
    pool = np.array([I32_MIN, I32_MIN + 1, I32_MIN + 2, I32_MAX, I32_MAX - 1, I32_MAX - 2, -1, 0, 1],
                    dtype=np.int64)
    vals = []
    for c in range(2):
        v = pool[g.integers(0, len(pool), size=n)]
        # a third of the rows lean positive or negative by group parity, so that
        # group sums run far past 2^31 in both directions
        lean = g.random(n) < 0.33
        v[lean & (keys % 2 == 0)] = I32_MAX
        v[lean & (keys % 2 == 1)] = I32_MIN
        vals.append(v.astype(np.int32))
    # group g_card: only INT32_MAX; group g_card + 1: only INT32_MIN;
    # groups g_card + 2 and g_card + 3: one row each
    extra_k = np.array([g_card] * 50 + [g_card + 1] * 50 + [g_card + 2, g_card + 3], dtype=np.int32)
    extra_v = np.array([I32_MAX] * 50 + [I32_MIN] * 50 + [I32_MIN, I32_MAX], dtype=np.int32)
    pos = g.integers(0, n + 1, size=len(extra_k))
    keys = np.insert(keys, pos, extra_k)
    vals = [np.insert(v, pos, extra_v) for v in vals]
    return keys, vals


AGGS = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]


def _compare(keys, res, want, what):
    from gpu_util import host
    gk = host(keys)
    order = np.argsort(gk, kind="stable")
    np.testing.assert_array_equal(gk[order], want["key"], err_msg=what)
    np.testing.assert_array_equal(host(res[0])[order], want["count"], err_msg=what)
    for c, (si, mi, xi) in enumerate([(1, 2, 3), (4, 5, 6)]):
        np.testing.assert_array_equal(host(res[si])[order], want["sum"][c], err_msg=what)
        np.testing.assert_array_equal(host(res[mi])[order], want["min"][c], err_msg=what)
        np.testing.assert_array_equal(host(res[xi])[order], want["max"][c], err_msg=what)


@pytest.mark.parametrize("alpha", [0.0, 1.1])
@pytest.mark.parametrize("g_card", [8, 3000, 200000])
def test_groupby_int32_extremes(alpha, g_card):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, say
    keys, vals = extreme_input((1 << 20) + 123, g_card, alpha, seed=5150 + g_card)
    want = oracle.groupby(keys, vals)
    big = np.abs(np.concatenate(want["sum"])).max()
    assert big > 2 ** 33, "the input must drive group sums past 32 bits"
    assert want["min"][0][want["key"] == g_card][0] == I32_MAX
    assert want["max"][0][want["key"] == g_card + 1][0] == I32_MIN
    dk, dv = dev(keys), [dev(v) for v in vals]
    for algo, mat in [("hash", "auto"), ("sort", "gftr"), ("sort", "gfur"), ("partition", "gftr"),
                      ("partition", "gfur"), ("sort_de", "gftr")]:
        say(f"extremes g={g_card} alpha={alpha}: {algo} {mat}")
        k, r = gj.groupby(dk, dv, AGGS, algo=algo, mat=mat)
        _compare(k, r, want, f"{algo}/{mat}")
    # tiny LDS budget: the hash group-by's global-atomic records
    k, r = gj.groupby(dk, dv, AGGS, algo="hash", lds_budget=256)
    _compare(k, r, want, "hash/global records")


@pytest.mark.parametrize("alpha", [0.0, 1.1])
def test_groupby_batch_int32_extremes(alpha):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    sizes = [5000, 1, 70000, 123457, 300]
    parts = [extreme_input(s, c, alpha, seed=600 + i) for i, (s, c) in
             enumerate(zip(sizes, [10, 1, 900, 20000, 5]))]
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]).tolist()
    keys = np.concatenate([p[0] for p in parts])
    vals = [np.concatenate([p[1][c] for p in parts]) for c in range(2)]
    say(f"batched group-by of {len(parts)} instances with int32 extremes, alpha={alpha}")
    dk, dv = dev(keys), [dev(v) for v in vals]
    for use_plan in (False, True):
        if use_plan:
            plan = gj.GroupByPlan(dk, dv, off, AGGS)
            plan.capture()
            plan.launch()
            gk, res, goff = plan.result()
        else:
            gk, res, goff = gj.groupby_batch(dk, dv, off, AGGS)
        for i, p in enumerate(parts):
            want = oracle.groupby(p[0], p[1])
            sl = slice(goff[i], goff[i + 1])
            _compare(gk[sl], [r[sl] for r in res], want, f"instance {i} plan={use_plan}")
        if use_plan:
            plan.close()
