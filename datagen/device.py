"""Device-side (torch CUDA Philox) generators for the 2^27..2^28-row workloads.

Same distributions as the host generators in this package, drawn on the GPU so
that multi-gigabyte inputs take seconds. This module draws random numbers only.
"""
from __future__ import annotations

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
