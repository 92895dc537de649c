"""Helpers for the GPU parity tests: host <-> device copies and canonical row order."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def canon(cols):
    """Rows sorted lexicographically: a join output as a multiset."""
    cols = [np.asarray(c) for c in cols]
    if len(cols[0]) == 0:
        return cols
    order = np.lexsort(tuple(reversed(cols)))
    return [c[order] for c in cols]


def say(msg: str):
    print(msg, flush=True)


_SM = (0x9E3779B97F4A7C15, 0xBF58476D1CE4E5B9, 0x94D049BB133111EB)


def unsplitmix64(z: np.ndarray) -> np.ndarray:
    """Inverse of the splitmix64 output function that widens 4-byte key values to
    8-byte keys: undoes each xor-shift and multiplies by the constants' inverses
    modulo 2^64. Returns the original values as int64."""
    g, c1, c2 = (np.uint64(c) for c in _SM)
    i1, i2 = np.uint64(pow(_SM[1], -1, 1 << 64)), np.uint64(pow(_SM[2], -1, 1 << 64))
    s = lambda v, k: v >> np.uint64(k)
    with np.errstate(over="ignore"):
        y = np.ascontiguousarray(z).view(np.uint64)
        y = y ^ s(y, 31) ^ s(y, 62)
        y = y * i2
        y = y ^ s(y, 27) ^ s(y, 54)
        y = y * i1
        y = y ^ s(y, 30) ^ s(y, 60)
        y = y - g
    return y.view(np.int64)
