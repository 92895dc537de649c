"""GPU parity for batches of independent joins: every instance's output equals
the oracle's join of that instance alone."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def make_batch(sizes, seed, key_bytes=4, many=False):
    parts = []
    for i, (nr, ns) in enumerate(sizes):
        if many:
            d = datagen.many_to_many_join(nr, ns, max(1, nr // 3), 2, 2, seed=seed + i, key_bytes=key_bytes)
        else:
            d = datagen.pk_fk_join(nr, ns, 2, 2, seed=seed + i, key_bytes=key_bytes,
                                   match_ratio=1.0 if i % 3 else 0.6)
        parts.append(d)
    cat = lambda xs, dt: np.concatenate(xs) if xs else np.zeros(0, dt)
    kd = np.int32 if key_bytes == 4 else np.int64
    b = {"r_key": cat([p["r_key"] for p in parts], kd), "s_key": cat([p["s_key"] for p in parts], kd),
         "r_pay": [cat([p["r_pay"][j] for p in parts], np.int32) for j in range(2)],
         "s_pay": [cat([p["s_pay"][j] for p in parts], np.int32) for j in range(2)],
         "r_off": np.concatenate([[0], np.cumsum([len(p["r_key"]) for p in parts])]),
         "s_off": np.concatenate([[0], np.cumsum([len(p["s_key"]) for p in parts])])}
    return parts, b


def check_batch(parts, b, mat):
    import paper_2312_00720_amd as gj
    from gpu_util import canon, dev, host, say
    say(f"batch of {len(parts)} instances, |R|={len(b['r_key'])} |S|={len(b['s_key'])} mat={mat}")
    k, rp, sp, off = gj.join_batch(dev(b["r_key"]), [dev(x) for x in b["r_pay"]], list(b["r_off"]),
                                   dev(b["s_key"]), [dev(x) for x in b["s_pay"]], list(b["s_off"]), mat=mat)
    cols = [host(k)] + [host(x) for x in rp] + [host(x) for x in sp]
    assert off[0] == 0 and off[-1] == len(cols[0])
    for i, p in enumerate(parts):
        want = oracle.join(p["r_key"], p["r_pay"], p["s_key"], p["s_pay"])
        got = [c[off[i]:off[i + 1]] for c in cols]
        assert len(got[0]) == len(want[0]), i
        for a, e in zip(canon(got), canon(want)):
            np.testing.assert_array_equal(a, e)


@pytest.mark.parametrize("mat", ["gftr", "gfur"])
def test_batch_uneven_instances(mat):
    g = datagen.rng(11)
    sizes = []
    for i in range(60):
        nr = int(round(2 ** g.uniform(0, 14)))
        sizes.append((nr, nr * int(g.integers(4, 17))))
    sizes[5] = (0, 100)      # empty build side
    sizes[17] = (300, 0)     # empty probe side
    sizes[30] = (1, 1)
    parts, b = make_batch(sizes, seed=1000)
    check_batch(parts, b, mat)


def test_batch_many_to_many_and_int64():
    g = datagen.rng(12)
    sizes = [(int(g.integers(1, 3000)), int(g.integers(1, 5000))) for _ in range(20)]
    parts, b = make_batch(sizes, seed=2000, many=True)
    check_batch(parts, b, "gftr")
    parts, b = make_batch(sizes, seed=3000, key_bytes=8)
    check_batch(parts, b, "gfur")


def test_batch_equals_single_calls():
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host
    sizes = [(5000, 40000), (200, 3000), (70000, 300000)]
    parts, b = make_batch(sizes, seed=4000)
    k, rp, sp, off = gj.join_batch(dev(b["r_key"]), [dev(x) for x in b["r_pay"]], list(b["r_off"]),
                                   dev(b["s_key"]), [dev(x) for x in b["s_pay"]], list(b["s_off"]), mat="gftr")
    for i, p in enumerate(parts):
        k1, r1, s1 = gj.join(dev(p["r_key"]), [dev(x) for x in p["r_pay"]], dev(p["s_key"]),
                             [dev(x) for x in p["s_pay"]], mat="gftr")
        got = [host(k)[off[i]:off[i + 1]]] + [host(x)[off[i]:off[i + 1]] for x in rp + sp]
        single = [host(k1)] + [host(x) for x in r1 + s1]
        assert oracle.rows_fingerprint(got) == oracle.rows_fingerprint(single)
