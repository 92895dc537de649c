"""Seeded synthetic inputs shaped like the paper's join and group-by workloads.

This module only draws random numbers. It holds none of the join or group-by
arithmetic, so both the CPU oracle and the GPU path can take their inputs from
it without sharing any of the method's code.

Workload shapes follow the paper's evaluation (Section 5):
  * joins: R holds primary keys 0..|R|-1 in random order, S holds foreign keys;
    payload columns are 4-byte integers (Section 5.1.1);
  * skew: foreign keys follow a Zipf law whose factor is varied (Section 5.1, data skew);
  * match ratio: a fraction of S rows has no partner in R (Section 5.1, match ratio);
  * group-by: keys uniform over {0..g-1} (or Zipf), value columns of 4-byte
    integers (Section 5.2.1).

Readings where the paper is silent:
  * unmatched foreign keys are drawn outside R's key range, and exactly
    round(mr*|S|) rows of S match, chosen by a seeded shuffle;
  * Zipf: P(rank = i) is proportional to i**-alpha for i = 1..n, sampled by
    inverse CDF over float64 cumulative weights; rank i maps to key i-1;
  * 8-byte keys: the splitmix64 output function (a published bijective mix) is
    applied to the 4-byte key values, so all 64 bits carry information;
  * group-by values are uniform on the closed range [-2^20, 2^20].

Two generator families are provided: host generators on NumPy's Philox bit
generator (small and medium sizes), and device generators on torch's CUDA
Philox generator for the 2^27..2^28-row workloads. They are separate recipes:
the same seed does not give the same arrays on both.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 231200720

INT32_MIN = -(2 ** 31)
INT32_MAX = 2 ** 31 - 1

_SM_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_SM_C1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_C2 = np.uint64(0x94D049BB133111EB)


def seed_for(config: int, variant: int = 0) -> int:
    """Seed of workload `config` (0-based), variant `variant`."""
    return SEED_BASE + 1000 * config + variant


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function (Steele, Lea, Flood 2014), bijective on uint64."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + _SM_GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _SM_C1
        z = (z ^ (z >> np.uint64(27))) * _SM_C2
        z = z ^ (z >> np.uint64(31))
    return z


def widen_keys(k32: np.ndarray) -> np.ndarray:
    """Map non-negative 4-byte key values to 8-byte keys (int64 bit patterns)."""
    return splitmix64(k32.astype(np.uint64)).view(np.int64)


def zipf_ranks(g: np.random.Generator, count: int, n: int, alpha: float) -> np.ndarray:
    """`count` draws of a rank in 1..n with P(i) ~ i**-alpha (alpha = 0: uniform)."""
    if count == 0:
        return np.zeros(0, dtype=np.int64)
    if alpha == 0.0:
        return g.integers(1, n + 1, size=count, dtype=np.int64)
    w = np.arange(1, n + 1, dtype=np.float64) ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = g.random(count)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, n).astype(np.int64)


def payload_columns(g: np.random.Generator, n: int, c: int) -> list[np.ndarray]:
    """c int32 columns uniform over the full int32 range."""
    return [g.integers(INT32_MIN, INT32_MAX + 1, size=n, dtype=np.int64).astype(np.int32)
            for _ in range(c)]


def pk_fk_join(n_r: int, n_s: int, c_r: int, c_s: int, seed: int, *,
               alpha: float = 0.0, match_ratio: float = 1.0,
               key_bytes: int = 4) -> dict:
    """Primary-key/foreign-key join inputs.

    R.key is a random permutation of 0..n_r-1 (mapped through splitmix64 for
    8-byte keys); S.key draws ranks from uniform (alpha = 0) or Zipf(alpha);
    exactly round(match_ratio * n_s) S rows match.
    """
    g = rng(seed)
    r32 = g.permutation(n_r).astype(np.int64)
    n_match = int(round(match_ratio * n_s))
    ranks = zipf_ranks(g, n_s, max(n_r, 1), alpha) if n_r > 0 else np.zeros(n_s, np.int64)
    s_val = ranks - 1
    matched = np.zeros(n_s, dtype=bool)
    if n_match > 0:
        matched[g.permutation(n_s)[:n_match]] = True
    n_un = n_s - n_match
    if key_bytes == 4:
        un = g.integers(n_r, INT32_MAX + 1, size=n_un, dtype=np.int64)
    else:
        un = g.integers(n_r, 2 ** 40, size=n_un, dtype=np.int64)
    s_val = s_val.copy()
    s_val[~matched] = un
    r_pay = payload_columns(g, n_r, c_r)
    s_pay = payload_columns(g, n_s, c_s)
    if key_bytes == 4:
        rk = r32.astype(np.int32)
        sk = s_val.astype(np.int32)
    elif key_bytes == 8:
        rk = widen_keys(r32)
        sk = widen_keys(s_val)
    else:
        raise ValueError("key_bytes must be 4 or 8")
    return {"r_key": rk, "r_pay": r_pay, "s_key": sk, "s_pay": s_pay,
            "n_match": n_match}


def many_to_many_join(n_r: int, n_s: int, n_keys: int, c_r: int, c_s: int,
                      seed: int, key_bytes: int = 4) -> dict:
    """Both sides draw keys uniformly from a set of n_keys unique values
    (the paper's many-to-many experiment, Section 5.1)."""
    g = rng(seed)
    rk = g.integers(0, n_keys, size=n_r, dtype=np.int64)
    sk = g.integers(0, n_keys, size=n_s, dtype=np.int64)
    r_pay = payload_columns(g, n_r, c_r)
    s_pay = payload_columns(g, n_s, c_s)
    if key_bytes == 4:
        rk, sk = rk.astype(np.int32), sk.astype(np.int32)
    else:
        rk, sk = widen_keys(rk), widen_keys(sk)
    return {"r_key": rk, "r_pay": r_pay, "s_key": sk, "s_pay": s_pay}


def groupby_input(n: int, g_card: int, n_vals: int, seed: int, *,
                  alpha: float = 0.0, key_bytes: int = 4,
                  lo: int = -(2 ** 20), hi: int = 2 ** 20) -> dict:
    """Group-by inputs: keys over {0..g-1} (uniform or Zipf(alpha) on ranks),
    n_vals int32 value columns uniform on [lo, hi]."""
    g = rng(seed)
    keys = zipf_ranks(g, n, g_card, alpha) - 1
    vals = [g.integers(lo, hi + 1, size=n, dtype=np.int64).astype(np.int32)
            for _ in range(n_vals)]
    if key_bytes == 4:
        k = keys.astype(np.int32)
    else:
        k = widen_keys(keys)
    return {"key": k, "vals": vals}


def raw_keys(n: int, seed: int, key_bytes: int = 4, lo=None, hi=None) -> np.ndarray:
    """Keys uniform over [lo, hi] (default: the full signed range)."""
    g = rng(seed)
    if key_bytes == 4:
        lo = INT32_MIN if lo is None else lo
        hi = INT32_MAX if hi is None else hi
        return g.integers(lo, hi + 1, size=n, dtype=np.int64).astype(np.int32)
    lo = -(2 ** 63) if lo is None else lo
    hi = 2 ** 63 - 1 if hi is None else hi
    return g.integers(lo, hi, size=n, dtype=np.int64, endpoint=True)


def batch_sizes(n: int, seed: int, lo_log2: float = 8.0, hi_log2: float = 20.0, m_lo: int = 4, m_hi: int = 16):
    """Instance sizes of a join batch: |R_i| = round(2^U(lo, hi)) and
    |S_i| = m_i |R_i| with m_i uniform over {m_lo..m_hi}."""
    g = rng(seed)
    r = np.rint(2.0 ** g.uniform(lo_log2, hi_log2, size=n)).astype(np.int64)
    m = g.integers(m_lo, m_hi + 1, size=n)
    return r, r * m
