"""GPU parity at the benchmark's full sizes, in the configuration bench.py times.

Join: |R| = 2^27, |S| = 2^28, 4 + 4 int32 payloads, uniform FKs, match ratio
100%, GFTR. Every output row is checked against the PK-FK closed form (R keys are
a permutation, so each row's R payloads are R.p[inv[key]]), and the multiset of
(key, S payloads) is checked against S with the oracle's order-independent
fingerprint.

Group-by: N = 2^28 keys over 2^16 values, 2 value columns, partition-based
GFTR. COUNT and SUM are checked against bincount closed forms (SUM exact in
float64 since |sum| < 2^53), MIN and MAX against scatter-reduce on the CPU.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def test_join_full_size_gftr():
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import say
    n_r, n_s = 1 << 27, 1 << 28
    say("full-size join: generating")
    d = dd.pk_fk_join(n_r, n_s, 4, 4, seed=datagen.seed_for(1))
    say("full-size join: running gj.join (gftr)")
    k, rp, sp = gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat="gftr")
    torch.cuda.synchronize()
    assert k.numel() == n_s
    say("full-size join: checking R payloads by the closed form")
    rk = d["r_key"].cpu().numpy()
    inv = np.empty(n_r, dtype=np.int64)
    inv[rk] = np.arange(n_r, dtype=np.int64)
    tk = k.cpu().numpy()
    assert tk.min() >= 0 and tk.max() < n_r
    ridx = inv[tk]
    for j in range(4):
        np.testing.assert_array_equal(rp[j].cpu().numpy(), d["r_pay"][j].cpu().numpy()[ridx])
    del ridx, inv
    say("full-size join: fingerprint of (key, S payloads)")
    got = oracle.rows_fingerprint([tk] + [x.cpu().numpy() for x in sp])
    want = oracle.rows_fingerprint([d["s_key"].cpu().numpy()] + [x.cpu().numpy() for x in d["s_pay"]])
    assert got == want


def test_groupby_full_size_partition():
    import torch
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    from gpu_util import say
    n, g = 1 << 28, 1 << 16
    say("full-size group-by: generating")
    d = dd.groupby_input(n, g, 2, seed=datagen.seed_for(2, 16))
    aggs = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]
    say("full-size group-by: running gj.groupby (partition, gftr)")
    keys, res = gj.groupby(d["key"], d["vals"], aggs, algo="partition", mat="gftr")
    torch.cuda.synchronize()
    k = d["key"].cpu().numpy().astype(np.int64)
    present = np.nonzero(np.bincount(k, minlength=g))[0]
    gk = keys.cpu().numpy().astype(np.int64)
    order = np.argsort(gk)
    np.testing.assert_array_equal(gk[order], present)
    say("full-size group-by: closed forms")
    cnt = np.bincount(k, minlength=g)[present]
    np.testing.assert_array_equal(res[0].cpu().numpy()[order], cnt)
    kt = torch.from_numpy(k)
    for c, (si, mi, xi) in enumerate([(1, 2, 3), (4, 5, 6)]):
        v = d["vals"][c].cpu().numpy()
        s = np.bincount(k, weights=v.astype(np.float64), minlength=g)[present]
        np.testing.assert_array_equal(res[si].cpu().numpy()[order], s.astype(np.int64))
        vt = torch.from_numpy(v.astype(np.int64))
        mn = torch.full((g,), 2**31 - 1, dtype=torch.int64).scatter_reduce(0, kt, vt, "amin")
        mx = torch.full((g,), -2**31, dtype=torch.int64).scatter_reduce(0, kt, vt, "amax")
        np.testing.assert_array_equal(res[mi].cpu().numpy()[order], mn.numpy()[present])
        np.testing.assert_array_equal(res[xi].cpu().numpy()[order], mx.numpy()[present])
