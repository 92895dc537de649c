"""Checks of the seeded input generators (shapes and distributions only)."""
import numpy as np

import datagen


def test_deterministic_per_seed():
    a = datagen.pk_fk_join(1000, 3000, 2, 2, seed=5, alpha=0.5, match_ratio=0.5)
    b = datagen.pk_fk_join(1000, 3000, 2, 2, seed=5, alpha=0.5, match_ratio=0.5)
    c = datagen.pk_fk_join(1000, 3000, 2, 2, seed=6, alpha=0.5, match_ratio=0.5)
    assert np.array_equal(a["s_key"], b["s_key"]) and np.array_equal(a["r_pay"][1], b["r_pay"][1])
    assert not np.array_equal(a["s_key"], c["s_key"])


def test_pk_is_permutation_and_match_count_exact():
    n_r, n_s = 4096, 10000
    for mr in (1.0, 0.5, 0.3, 0.0):
        d = datagen.pk_fk_join(n_r, n_s, 1, 1, seed=1, match_ratio=mr)
        assert np.array_equal(np.sort(d["r_key"]), np.arange(n_r, dtype=np.int32))
        assert int(np.isin(d["s_key"], d["r_key"]).sum()) == int(round(mr * n_s))
        un = d["s_key"][~np.isin(d["s_key"], d["r_key"])]
        assert np.all(un >= n_r)


def test_int64_keys_are_bijective_images():
    d = datagen.pk_fk_join(5000, 9000, 1, 1, seed=2, key_bytes=8, match_ratio=0.5)
    assert d["r_key"].dtype == np.int64 and len(np.unique(d["r_key"])) == 5000
    assert int(np.isin(d["s_key"], d["r_key"]).sum()) == 4500


def test_zipf_rank_frequencies():
    g = datagen.rng(3)
    n, cnt, alpha = 1000, 1 << 20, 1.0
    r = datagen.zipf_ranks(g, cnt, n, alpha)
    h = np.bincount(r, minlength=n + 1)[1:]
    p = np.arange(1, n + 1, dtype=np.float64) ** -alpha
    p /= p.sum()
    # chi-square over the 50 hottest ranks plus the remainder, loose bound
    exp = np.concatenate([p[:50], [p[50:].sum()]]) * cnt
    obs = np.concatenate([h[:50], [h[50:].sum()]])
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 120.0  # 50 degrees of freedom; p ~ 1e-7 at 120
    assert r.min() >= 1 and r.max() <= n
