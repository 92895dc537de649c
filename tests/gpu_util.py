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
