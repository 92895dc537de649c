"""The learned selector (a15): trained on the GPU by the library's own kernels on
the committed timings of seeded workloads, the network's held-out regret is
below the cost model's (what it gains over the method without it), and an
automatic choice never changes a result."""
import os

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "paper_2312_00720_amd", "selector_data.npz")


def test_trained_network_beats_cost_model():
    """Trained as selector.py trains it (both feature views), scored on the
    held-out workloads' product-path features: the vectors gj_join and
    gj_groupby compute by themselves, without hints."""
    import paper_2312_00720_amd as gj
    from paper_2312_00720_amd import selector
    from gpu_util import say
    z = selector.load_data(DATA)
    say(f"selector: {len(z['Xtr'])} training and {len(z['Xte'])} held-out workloads")
    theta = selector.train(np.concatenate([z["Xtr"], z["Htr"]]), np.concatenate([z["Mtr"]] * 2),
                           np.concatenate([z["Ttr"]] * 2), steps=3000)
    assert np.isfinite(theta).all()
    rep = selector.evaluate_arrays(z["Xte"], z["Mte"], z["Tte"], theta)
    say(f"held-out regret: {rep}")
    assert rep["mlp"]["aggregate_pct"] < rep["cost_model"]["aggregate_pct"]
    assert rep["mlp"]["mean_pct"] < rep["cost_model"]["mean_pct"]
    assert rep["mlp"]["aggregate_pct"] >= 0.0
    gj.selector_set_weights(None)
    gj._load_shipped_weights(gj.lib())


def test_automatic_choice_never_changes_results():
    import paper_2312_00720_amd as gj
    from gpu_util import canon, dev, host
    d = datagen.pk_fk_join(30000, 200000, 2, 2, seed=71, match_ratio=0.4)
    want = canon(oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"]))
    for weights in ("shipped", None):
        if weights is None:
            gj.selector_set_weights(None)
        k, rp, sp = gj.join(dev(d["r_key"]), [dev(x) for x in d["r_pay"]], dev(d["s_key"]),
                            [dev(x) for x in d["s_pay"]], mat="auto")
        for a, e in zip(canon([host(k)] + [host(x) for x in rp + sp]), want):
            np.testing.assert_array_equal(a, e)
        g = datagen.groupby_input(100000, 3000, 2, seed=72)
        o = oracle.groupby(g["key"], g["vals"])
        keys, cols = gj.groupby(dev(g["key"]), [dev(v) for v in g["vals"]], [(0, "count"), (1, "max")], algo="auto")
        keys = host(keys)
        order = np.argsort(keys, kind="stable")
        np.testing.assert_array_equal(keys[order], o["key"])
        np.testing.assert_array_equal(host(cols[0])[order], o["count"])
        np.testing.assert_array_equal(host(cols[1])[order], o["max"][1])
    gj._load_shipped_weights(gj.lib())
