"""Device-side (torch CUDA Philox) generators for the 2^27..2^28-row workloads.

Same distributions as the host generators in this package, drawn on the GPU so
that multi-gigabyte inputs take seconds. This module draws random numbers only.
"""
from __future__ import annotations

import numpy as np
import torch

INT32_MIN = -(2 ** 31)
INT32_MAX = 2 ** 31 - 1


def generator(seed: int, device="cuda") -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def payloads(g: torch.Generator, n: int, c: int, device="cuda") -> list:
    """c int32 columns uniform over the full int32 range."""
    return [torch.randint(INT32_MIN, INT32_MAX, (n,), generator=g, device=device,
                          dtype=torch.int64).to(torch.int32) for _ in range(c)]


def zipf_ranks(g: torch.Generator, count: int, n: int, alpha: float, device="cuda") -> torch.Tensor:
    """`count` ranks in 1..n with P(i) ~ i**-alpha (alpha = 0: uniform), int64."""
    if alpha == 0.0:
        return torch.randint(1, n + 1, (count,), generator=g, device=device, dtype=torch.int64)
    w = torch.arange(1, n + 1, device=device, dtype=torch.float64).pow_(-alpha)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    del w
    u = torch.rand(count, generator=g, device=device, dtype=torch.float64)
    r = torch.searchsorted(cdf, u, right=True) + 1
    return r.clamp_(max=n)


def _splitmix64(x: torch.Tensor) -> torch.Tensor:
    """splitmix64 output function on int64 tensors (two's-complement wraparound)."""
    def c(v):
        return v - (1 << 64) if v >= (1 << 63) else v
    z = x + c(0x9E3779B97F4A7C15)
    z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * c(0xBF58476D1CE4E5B9)
    z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * c(0x94D049BB133111EB)
    return z ^ ((z >> 31) & ((1 << 33) - 1))


def pk_fk_join(n_r: int, n_s: int, c_r: int, c_s: int, seed: int, *, alpha: float = 0.0,
               match_ratio: float = 1.0, key_bytes: int = 4, device="cuda") -> dict:
    """PK-FK join inputs as device tensors (see datagen.pk_fk_join for the recipe)."""
    g = generator(seed, device)
    r = torch.randperm(n_r, generator=g, device=device, dtype=torch.int64)
    s = zipf_ranks(g, n_s, n_r, alpha, device) - 1
    n_match = int(round(match_ratio * n_s))
    if n_match < n_s:
        un_idx = torch.randperm(n_s, generator=g, device=device)[n_match:]
        hi = INT32_MAX + 1 if key_bytes == 4 else 2 ** 40
        s[un_idx] = torch.randint(n_r, hi, (n_s - n_match,), generator=g, device=device,
                                  dtype=torch.int64)
        del un_idx
    r_pay = payloads(g, n_r, c_r, device)
    s_pay = payloads(g, n_s, c_s, device)
    if key_bytes == 4:
        rk, sk = r.to(torch.int32), s.to(torch.int32)
    else:
        rk, sk = _splitmix64(r), _splitmix64(s)
    return {"r_key": rk, "r_pay": r_pay, "s_key": sk, "s_pay": s_pay, "n_match": n_match}


def groupby_input(n: int, g_card: int, n_vals: int, seed: int, *, alpha: float = 0.0,
                  lo: int = -(2 ** 20), hi: int = 2 ** 20, device="cuda") -> dict:
    """Group-by inputs as device tensors (see datagen.groupby_input)."""
    g = generator(seed, device)
    k = (zipf_ranks(g, n, g_card, alpha, device) - 1).to(torch.int32)
    vals = [torch.randint(lo, hi + 1, (n,), generator=g, device=device, dtype=torch.int64)
            .to(torch.int32) for _ in range(n_vals)]
    return {"key": k, "vals": vals}


def join_batch(r_sizes, s_sizes, c: int, seed: int, device="cuda", chunk_rows: int = 1 << 28) -> dict:
    """A batch of independent PK-FK joins, stored back to back: instance i has
    R_i.key a random permutation of 0..|R_i|-1 and S_i.key uniform over R_i's
    keys (every S row matches), c int32 payload columns per side uniform over the
    full range. Drawn in chunks of instances so temporaries stay small."""
    import numpy as np
    r_sizes = np.asarray(r_sizes, dtype=np.int64)
    s_sizes = np.asarray(s_sizes, dtype=np.int64)
    n = len(r_sizes)
    ro = np.concatenate([[0], np.cumsum(r_sizes)])
    so = np.concatenate([[0], np.cumsum(s_sizes)])
    g = generator(seed, device)
    r_key = torch.empty(int(ro[-1]), dtype=torch.int32, device=device)
    s_key = torch.empty(int(so[-1]), dtype=torch.int32, device=device)
    i = 0
    while i < n:
        j, rows = i, 0
        while j < n and (j == i or rows + int(s_sizes[j]) <= chunk_rows):
            rows += int(s_sizes[j])
            j += 1
        rs = torch.from_numpy(r_sizes[i:j]).to(device)
        ss = torch.from_numpy(s_sizes[i:j]).to(device)
        m = torch.arange(j - i, device=device)
        # R: local row ids, shuffled within each instance
        inst = torch.repeat_interleave(m, rs)
        start = torch.from_numpy(ro[i:j] - ro[i]).to(device)
        local = torch.arange(int(ro[j] - ro[i]), device=device) - start[inst]
        rnd = torch.randint(0, 1 << 31, (local.numel(),), generator=g, device=device, dtype=torch.int64)
        order = torch.argsort(inst * (1 << 31) + rnd)
        r_key[int(ro[i]):int(ro[j])] = local[order].to(torch.int32)
        del inst, local, rnd, order
        # S: uniform over the instance's keys
        sinst = torch.repeat_interleave(m, ss)
        u = torch.rand(int(so[j] - so[i]), generator=g, device=device, dtype=torch.float64)
        k = torch.minimum((u * rs[sinst]).to(torch.int64), rs[sinst] - 1)
        s_key[int(so[i]):int(so[j])] = k.to(torch.int32)
        del sinst, u, k
        i = j
    r_pay = payloads(g, int(ro[-1]), c, device)
    s_pay = payloads(g, int(so[-1]), c, device)
    return {"r_key": r_key, "r_pay": r_pay, "s_key": s_key, "s_pay": s_pay,
            "r_off": [int(x) for x in ro], "s_off": [int(x) for x in so]}


def groupby_batch(sizes, cards, n_vals: int, seed: int, *, lo: int = -(2 ** 20), hi: int = 2 ** 20,
                  device="cuda") -> dict:
    """A batch of independent group-bys stored back to back: instance i has
    sizes[i] rows whose int32 keys are uniform over 0..cards[i]-1, and n_vals int32
    value columns uniform in [lo, hi]. Returns the columns and the host offsets."""
    g = generator(seed, device)
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    n = int(off[-1])
    card = torch.repeat_interleave(torch.as_tensor(np.asarray(cards, dtype=np.int64), device=device),
                                   torch.as_tensor(sizes, device=device))
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    key = torch.minimum((u * card).to(torch.int64), card - 1).to(torch.int32)
    del u, card
    vals = [torch.randint(lo, hi + 1, (n,), generator=g, device=device, dtype=torch.int64)
            .to(torch.int32) for _ in range(n_vals)]
    return {"key": key, "vals": vals, "off": [int(x) for x in off]}
