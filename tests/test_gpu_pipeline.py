"""GPU parity for the join followed by a group-by on its output (the operator
pair that motivates the paper, Section 1): T = R |><| S, then group T by an R
payload column and aggregate an S payload column."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("algo", ["partition", "hash", "sort"])
@pytest.mark.parametrize("mat", ["gftr", "gfur"])
def test_join_then_groupby(algo, mat):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    n_r, n_s = 1 << 14, 1 << 18
    d = datagen.pk_fk_join(n_r, n_s, 1, 1, seed=datagen.seed_for(2, 77))
    g = datagen.rng(78)
    # the R payload that is grouped on has about 2^10 distinct values
    d["r_pay"] = [g.integers(0, 1 << 10, size=n_r).astype(np.int32)]
    d["s_pay"] = [g.integers(-2**20, 2**20 + 1, size=n_s).astype(np.int32)]
    say(f"pipeline join({mat}) -> groupby({algo})")
    k, rp, sp = gj.join(dev(d["r_key"]), [dev(x) for x in d["r_pay"]], dev(d["s_key"]),
                        [dev(x) for x in d["s_pay"]], mat=mat)
    aggs = [(0, "count"), (0, "sum"), (0, "min"), (0, "max")]
    gk, res = gj.groupby(rp[0], [sp[0]], aggs, algo=algo, mat=mat if algo != "hash" else "auto")
    t = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    o = oracle.groupby(t[1], [t[2]])
    gk = host(gk)
    order = np.argsort(gk, kind="stable")
    np.testing.assert_array_equal(gk[order], o["key"])
    np.testing.assert_array_equal(host(res[0])[order], o["count"])
    np.testing.assert_array_equal(host(res[1])[order], o["sum"][0])
    np.testing.assert_array_equal(host(res[2])[order], o["min"][0])
    np.testing.assert_array_equal(host(res[3])[order], o["max"][0])
