"""Training and evaluation of the algorithm selector on the GPU.

1. Sample seeded workloads over the feature ranges (joins: log2|R| in [10, 24],
   |S|/|R| in [1, 16], 1-8 payload columns, 4- or 8-byte keys, Zipf factor in
   [0, 1.2], match ratio in [0.05, 1]; group-bys: log2 N in [16, 26],
   log2 g in [2, min(24, log2 N)], 1-8 value columns).
2. Time every valid algorithm of each workload with libgj (median of 5 runs
   after one warm-up). Timing can be split into parts (`--part i --parts K`),
   each saving its own file, and merged afterwards (`--merge`).
3. Train the 12-64-64-5 network with libgj's own HIP gradient and Adam kernels;
   the label is the fastest class.
4. Report regret on held-out workloads: t(choice) / t(best) - 1, for the network,
   the cost model, the paper's heuristics (the group-by decision tree of
   Section 5.2 and the join rule of Section 7) and fixed choices.

Usage: python -m paper_2312_00720_amd.selector --train 20000 --test 2000 --out DIR
       [--part i --parts K]   time only part i of K of both sets
       [--merge PARTS_DIR --parts K]   merge the timed parts, train and report
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

import paper_2312_00720_amd as gj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLASSES = gj.CLASSES
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.f32")


def sample(n: int, seed: int) -> list[dict]:
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        if g.uniform() < 0.5:
            lr = g.uniform(10, 24)
            ratio = g.uniform(1, 16)
            ls = lr + math.log2(ratio)
            out.append(dict(kind="join", log_r=lr, log_s=ls, cr=int(g.integers(1, 9)), cs=int(g.integers(1, 9)),
                            kb=int(g.choice([4, 8])), alpha=float(g.choice([0.0, g.uniform(0, 1.2)])),
                            mr=float(g.uniform(0.05, 1.0)), seed=seed * 100000 + i))
        else:
            ln = g.uniform(16, 26)
            lg = g.uniform(2, min(24.0, ln))
            out.append(dict(kind="groupby", log_n=ln, log_g=lg, nv=int(g.integers(1, 9)), kb=int(g.choice([4, 8])),
                            alpha=float(g.choice([0.0, g.uniform(0, 1.2)])), seed=seed * 100000 + i))
    return out


def features(w: dict) -> list[float]:
    if w["kind"] == "join":
        nr, ns = 2 ** w["log_r"], 2 ** w["log_s"]
        return [1.0, w["log_r"] / 32, w["log_s"] / 32, w["log_r"] / 32, w["kb"] / 8, w["cr"] / 8, w["cs"] / 8,
                w["alpha"] / 1.2, w["mr"], (w["log_s"] - w["log_r"]) / 32, math.log2(max(1.0, w["mr"] * ns)) / 32,
                math.log2(nr * (w["kb"] + 4 * w["cr"]) + ns * (w["kb"] + 4 * w["cs"])) / 48]
    n = 2 ** w["log_n"]
    return [0.0, w["log_n"] / 32, 0.0, w["log_g"] / 32, w["kb"] / 8, w["nv"] / 8, 0.0, w["alpha"] / 1.2, 1.0,
            (w["log_n"] - w["log_g"]) / 32, w["log_g"] / 32, math.log2(n * (w["kb"] + 4 * w["nv"])) / 48]


def valid(w: dict) -> list[int]:
    return [0, 1] if w["kind"] == "join" else [2, 3, 4]


def _inputs(w: dict):
    import datagen.device as dd
    if w["kind"] == "join":
        d = dd.pk_fk_join(int(2 ** w["log_r"]), int(2 ** w["log_s"]), w["cr"], w["cs"], w["seed"],
                          alpha=w["alpha"], match_ratio=w["mr"], key_bytes=w["kb"])
        return d
    d = dd.groupby_input(int(2 ** w["log_n"]), max(1, int(2 ** w["log_g"])), w["nv"], w["seed"], alpha=w["alpha"])
    if w["kb"] == 8:
        d["key"] = d["key"].to(torch.int64) * 0x9E3779B1  # spread 8-byte keys over all bits
    return d


def run(w: dict, d, cls: int):
    if w["kind"] == "join":
        return gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat=CLASSES[cls])
    # COUNT, then SUM of every value column and MAX of the first seven (16 aggregates at most)
    aggs = [(0, "count")] + [(c, "sum") for c in range(w["nv"])] + [(c, "max") for c in range(min(w["nv"], 7))]
    algo = CLASSES[cls]
    return gj.groupby(d["key"], d["vals"], aggs, algo=algo, mat="gftr" if algo != "hash" else "auto")


def time_workload(w: dict, reps: int = 5) -> list[float]:
    d = _inputs(w)
    t = [math.inf] * 5
    for c in valid(w):
        try:
            out = run(w, d, c)  # warm-up
        except RuntimeError as e:  # a library error (e.g. out of memory): the class stays untimed
            print(f"[selector] {CLASSES[c]} failed on {w}: {e}", flush=True)
            continue
        del out
        samples = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = run(w, d, c)
            torch.cuda.synchronize()
            samples.append(time.perf_counter() - t0)
            del out
        t[c] = float(np.median(samples))
    del d
    return t


def build(ws: list[dict], log_every: int = 100) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    X = np.array([features(w) for w in ws], np.float32).reshape(len(ws), 12)
    M = np.zeros((len(ws), 5), np.float32)
    T = np.full((len(ws), 5), np.inf)
    t0 = time.time()
    for i, w in enumerate(ws):
        M[i, valid(w)] = 1
        T[i] = time_workload(w)
        if (i + 1) % log_every == 0:
            print(f"[selector] timed {i + 1}/{len(ws)} ({time.time() - t0:.0f} s)", flush=True)
    return X, M, T


def part_slice(n: int, part: int, parts: int) -> slice:
    return slice(n * part // parts, n * (part + 1) // parts)


def init_params(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (He et al. 2015), zero biases, in the flat layout of gj.h."""
    g = np.random.Generator(np.random.Philox(seed))
    parts = []
    for shape in [(64, 12), (64,), (64, 64), (64,), (5, 64), (5,)]:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / shape[1])
            parts.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def train(X, M, T, steps: int = 3000, batch: int = 256, lr: float = 3e-3, seed: int = 7) -> np.ndarray:
    y = np.argmin(np.where(M > 0, T, np.inf), axis=1).astype(np.int32)
    dev = "cuda"
    P = torch.tensor(init_params(seed), dtype=torch.float32, device=dev)
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    Xd = torch.tensor(X, device=dev)
    Md = torch.tensor(M, device=dev)
    Yd = torch.tensor(y, device=dev)
    g = np.random.default_rng(seed)
    for t in range(1, steps + 1):
        b = torch.tensor(g.choice(len(X), min(batch, len(X)), replace=False), device=dev)
        _, grad = gj.mlp_grad(P, Xd[b].contiguous(), Md[b].contiguous(), Yd[b].contiguous())
        gj.mlp_adam(P, grad, m, v, t, lr=lr)
    return P.cpu().numpy()


def heuristic_choice(w: dict) -> int:
    """The paper's rules: joins use GFTR when mr >= 25%, the FKs are skewed or the
    keys are 8 bytes (Section 7); group-bys follow the decision tree (Section 5.2):
    HGB when its aggregates fit in shared memory, else sort for high skew, else
    PGB-TR."""
    if w["kind"] == "join":
        return 0 if (w["mr"] >= 0.25 or w["alpha"] >= 1.0 or w["kb"] == 8) else 1
    rec = 8 + 16 * w["nv"]
    if 2 ** w["log_g"] * rec <= 65536:
        return 2
    return 3 if w["alpha"] >= 1.0 else 4


def regret(T: np.ndarray, M: np.ndarray, choice: np.ndarray) -> dict:
    Tv = np.where(M > 0, T, np.inf)
    best = Tv.min(axis=1)
    tc = T[np.arange(len(T)), choice]
    r = tc / best - 1.0
    return {"mean_pct": float(100 * r.mean()), "p95_pct": float(100 * np.percentile(r, 95)),
            "aggregate_pct": float(100 * (tc.sum() / best.sum() - 1.0)), "best_picked_pct": float(100 * np.mean(r == 0))}


def evaluate_arrays(X, M, T, theta) -> dict:
    """Regret of the network (theta), the cost model, and a fixed choice, from
    feature and timing arrays alone."""
    gj.selector_set_weights(theta)
    mlp_c = np.array([gj.select(x, 0 if m[0] else 1)[0] for x, m in zip(X, M)])
    gj.selector_set_weights(None)
    cm_c = np.array([gj.select(x, 0 if m[0] else 1)[0] for x, m in zip(X, M)])
    fixed = np.array([0 if m[0] else 4 for m in M])
    rep = {"mlp": regret(T, M, mlp_c), "cost_model": regret(T, M, cm_c), "always_gftr_pgb": regret(T, M, fixed)}
    t_mlp = T[np.arange(len(T)), mlp_c].sum()
    t_cm = T[np.arange(len(T)), cm_c].sum()
    rep["mlp_vs_cost_model_pct"] = float(100 * (t_mlp / t_cm - 1.0))
    rep["n"] = int(len(X))
    return rep


def evaluate(ws, X, M, T, theta) -> dict:
    gj.selector_set_weights(theta)
    mlp_c = np.array([gj.select(x, 0 if m[0] else 1)[0] for x, m in zip(X, M)])
    gj.selector_set_weights(None)
    cm_c = np.array([gj.select(x, 0 if m[0] else 1)[0] for x, m in zip(X, M)])
    he_c = np.array([heuristic_choice(w) for w in ws])
    fixed = np.array([0 if w["kind"] == "join" else 4 for w in ws])
    rep = {"mlp": regret(T, M, mlp_c), "cost_model": regret(T, M, cm_c), "paper_heuristics": regret(T, M, he_c),
           "always_gftr_pgb": regret(T, M, fixed)}
    t_mlp = T[np.arange(len(T)), mlp_c].sum()
    t_cm = T[np.arange(len(T)), cm_c].sum()
    rep["mlp_vs_cost_model_pct"] = float(100 * (t_mlp / t_cm - 1.0))
    rep["n"] = int(len(ws))
    return rep


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default="gpurun_out/selector")
    ap.add_argument("--data", default=None, help="reuse timings from this .npz (no re-timing)")
    ap.add_argument("--part", type=int, default=None)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--merge", default=None, metavar="DIR", help="merge the timed parts found in DIR")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    tr, te = sample(args.train, 1), sample(args.test, 2)
    if args.part is not None:
        a, b = part_slice(len(tr), args.part, args.parts), part_slice(len(te), args.part, args.parts)
        print(f"[selector] part {args.part}/{args.parts}: train {a.start}..{a.stop}, test {b.start}..{b.stop}",
              flush=True)
        Xtr, Mtr, Ttr = build(tr[a])
        Xte, Mte, Tte = build(te[b])
        np.savez(os.path.join(args.out, f"selector_part{args.part:03d}of{args.parts:03d}.npz"), Xtr=Xtr, Mtr=Mtr,
                 Ttr=Ttr, Xte=Xte, Mte=Mte, Tte=Tte)
        return 0
    if args.merge:
        z = [np.load(os.path.join(args.merge, f"selector_part{i:03d}of{args.parts:03d}.npz"))
             for i in range(args.parts)]
        Xtr, Mtr, Ttr, Xte, Mte, Tte = (np.concatenate([q[k] for q in z]) for k in
                                        ("Xtr", "Mtr", "Ttr", "Xte", "Mte", "Tte"))
        np.savez(os.path.join(args.out, "selector_data.npz"), Xtr=Xtr, Mtr=Mtr, Ttr=Ttr, Xte=Xte, Mte=Mte, Tte=Tte)
    elif args.data:
        z = np.load(args.data)
        Xtr, Mtr, Ttr, Xte, Mte, Tte = (z[k] for k in ("Xtr", "Mtr", "Ttr", "Xte", "Mte", "Tte"))
    else:
        Xtr, Mtr, Ttr = build(tr)
        Xte, Mte, Tte = build(te)
        np.savez(os.path.join(args.out, "selector_data.npz"), Xtr=Xtr, Mtr=Mtr, Ttr=Ttr, Xte=Xte, Mte=Mte, Tte=Tte)
    theta = train(Xtr, Mtr, Ttr, steps=args.steps)
    theta.astype("<f4").tofile(os.path.join(args.out, "selector_weights.f32"))
    rep = {"train": evaluate(tr, Xtr, Mtr, Ttr, theta), "test": evaluate(te, Xte, Mte, Tte, theta)}
    with open(os.path.join(args.out, "selector_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps(rep), flush=True)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    sys.exit(main())
