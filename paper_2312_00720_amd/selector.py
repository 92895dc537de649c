"""Training and evaluation of the algorithm selector on the GPU.

1. Sample seeded workloads over the feature ranges (joins: log2|R| in [10, 24],
   |S|/|R| in [1, 16], 1-8 payload columns, 4- or 8-byte keys, Zipf factor in
   [0, 1.2], match ratio in [0.05, 1]; group-bys: log2 N in [16, 26],
   log2 g in [2, min(24, log2 N)], 1-8 value columns), plus (`--large`) sets of
   group-bys at log2 N in [26, 28], the grouped-aggregation benchmark's size.
2. Time every valid algorithm of each workload with libgj (median of 5 runs
   after one warm-up). Timing can be split into parts (`--part i --parts K`),
   each saving its own file, and merged afterwards (`--merge`).
3. Train the 12-64-64-7 network with libgj's own HIP gradient and Adam kernels
   on the feature vectors the library itself computes (gj_join_features,
   gj_groupby_features), both without hints and with the true match ratio and
   skew as hints; the label is the fastest class.
4. Report regret on held-out workloads: t(choice) / t(best) - 1, for the network,
   the cost model, the paper's heuristics (the group-by decision tree of
   Section 5.2 and the join rule of Section 7) and fixed choices, for both
   feature views, over all seven classes and over the first five.

Usage: python -m paper_2312_00720_amd.selector --train 20000 --test 2000 --out DIR
       [--part i --parts K]   time only part i of K of both sets
       [--large A,B --large-only --part i --parts K]   time part i of the extension sets
       [--merge PARTS_DIR --parts K [--large A,B]]   merge the timed parts, train and report
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
                            alpha=float(g.choice([0.0, g.uniform(0, 1.2)])), sparse=bool(g.uniform() < 0.5),
                            seed=seed * 100000 + i))
    return out


def sample_large(n: int, seed: int) -> list[dict]:
    """Group-bys at 2^26-2^28 rows (the size of the grouped-aggregation benchmark),
    timed as an extension of the main sets, whose row counts stop at 2^26."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ln = g.uniform(26, 28)
        lg = g.uniform(2, 24)
        out.append(dict(kind="groupby", log_n=ln, log_g=lg, nv=int(g.integers(1, 9)), kb=int(g.choice([4, 8])),
                        alpha=float(g.choice([0.0, g.uniform(0, 1.2)])), sparse=bool(g.uniform() < 0.5),
                        seed=seed * 100000 + i))
    return out


def valid(w: dict) -> list[int]:
    return list(gj.JOIN_CLASSES) if w["kind"] == "join" else list(gj.GROUPBY_CLASSES)


def _inputs(w: dict):
    import datagen.device as dd
    if w["kind"] == "join":
        d = dd.pk_fk_join(int(2 ** w["log_r"]), int(2 ** w["log_s"]), w["cr"], w["cs"], w["seed"],
                          alpha=w["alpha"], match_ratio=w["mr"], key_bytes=w["kb"])
        return d
    d = dd.groupby_input(int(2 ** w["log_n"]), max(1, int(2 ** w["log_g"])), w["nv"], w["seed"], alpha=w["alpha"])
    if w["kb"] == 8:
        d["key"] = d["key"].to(torch.int64) * 0x9E3779B1  # spread 8-byte keys over all bits
    elif w.get("sparse"):
        # an odd multiplier is a bijection modulo 2^32: the keys stay distinct and all 4 bytes vary
        d["key"] = ((d["key"].to(torch.int64) * 0x9E3779B1) & 0xFFFFFFFF).to(torch.int32)
    return d


def product_features(w: dict, d, hinted: bool) -> list[float]:
    """The feature vector the library's automatic choice computes for these
    inputs: without hints (what gj_join / gj_groupby see by themselves), or
    with the true match ratio and skew passed as hints."""
    if w["kind"] == "join":
        return gj.join_features(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"],
                                match_ratio_hint=w["mr"] if hinted else 0.0,
                                skew_hint=w["alpha"] if hinted else 0.0)
    return gj.groupby_features(d["key"], d["vals"], gb_aggs(w["nv"]), skew_hint=w["alpha"] if hinted else 0.0)


def gb_aggs(nv: int) -> list:
    """The aggregates a timed group-by computes: COUNT, then SUM of every value
    column and MAX of the first seven (16 aggregates at most)."""
    return [(0, "count")] + [(c, "sum") for c in range(nv)] + [(c, "max") for c in range(min(nv, 7))]


def run(w: dict, d, cls: int):
    if w["kind"] == "join":
        if cls == 6:
            return gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat="gftr", algo="smj")
        return gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat=CLASSES[cls], algo="phj")
    algo = CLASSES[cls]
    return gj.groupby(d["key"], d["vals"], gb_aggs(w["nv"]), algo=algo, mat="auto" if algo == "hash" else "gftr")


def time_workload(w: dict, reps: int = 5):
    """(median seconds per class, product features, hinted features)."""
    d = _inputs(w)
    t = [math.inf] * gj.N_CLASSES
    fp, fh = product_features(w, d, False), product_features(w, d, True)
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
    return t, fp, fh


def build(ws: list[dict], log_every: int = 100):
    """Timings T [n, classes], masks M, product features X and hinted features H."""
    C = gj.N_CLASSES
    X = np.zeros((len(ws), 12), np.float32)
    H = np.zeros((len(ws), 12), np.float32)
    M = np.zeros((len(ws), C), np.float32)
    T = np.full((len(ws), C), np.inf)
    t0 = time.time()
    for i, w in enumerate(ws):
        M[i, valid(w)] = 1
        T[i], X[i], H[i] = time_workload(w)
        if (i + 1) % log_every == 0:
            print(f"[selector] timed {i + 1}/{len(ws)} ({time.time() - t0:.0f} s)", flush=True)
    return X, H, M, T


def load_data(path: str) -> dict:
    """A timing set: Xtr/Htr/Mtr/Ttr and Xte/Hte/Mte/Tte. Sets timed before the
    sort-merge and dictionary-encoding classes existed have 5 class columns and
    no hinted features: the new classes are padded as untimed (masked out), and
    H repeats X."""
    z = np.load(path, allow_pickle=False)
    out = {}
    for part in ("tr", "te"):
        X, M, T = z["X" + part], z["M" + part], z["T" + part]
        if M.shape[1] < gj.N_CLASSES:
            pad = gj.N_CLASSES - M.shape[1]
            M = np.concatenate([M, np.zeros((len(M), pad), M.dtype)], axis=1)
            T = np.concatenate([T, np.full((len(T), pad), np.inf)], axis=1)
        out["X" + part], out["M" + part], out["T" + part] = X, M, T
        out["H" + part] = z["H" + part] if ("H" + part) in z.files else X
    return out


def part_slice(n: int, part: int, parts: int) -> slice:
    return slice(n * part // parts, n * (part + 1) // parts)


def init_params(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (He et al. 2015), zero biases, in the flat layout of gj.h."""
    g = np.random.Generator(np.random.Philox(seed))
    parts = []
    for shape in [(64, 12), (64,), (64, 64), (64,), (gj.N_CLASSES, 64), (gj.N_CLASSES,)]:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / shape[1])
            parts.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def heuristic_choice(w: dict) -> int:
    """The paper's rules: joins use GFTR when mr >= 25%, the FKs are skewed or the
    keys are 8 bytes (Section 7); group-bys follow the decision tree (Section 5.2):
    HGB when its aggregates fit in shared memory, else for high skew a sort-based
    group-by (with dictionary encoding when Table 2 says it pays: g < 2^15 for
    4-byte keys, g < 2^22 for 8-byte keys), else PGB-TR."""
    if w["kind"] == "join":
        return 0 if (w["mr"] >= 0.25 or w["alpha"] >= 1.0 or w["kb"] == 8) else 1
    rec = 8 + 16 * w["nv"]
    if 2 ** w["log_g"] * rec <= 65536:
        return 2
    if w["alpha"] >= 1.0:
        de_pays = w["log_g"] < (15 if w["kb"] == 4 else 22)
        return 5 if de_pays else 3
    return 4


def regret(T: np.ndarray, M: np.ndarray, choice: np.ndarray) -> dict:
    Tv = np.where(M > 0, T, np.inf)
    best = Tv.min(axis=1)
    tc = T[np.arange(len(T)), choice]
    r = tc / best - 1.0
    return {"mean_pct": float(100 * r.mean()), "p95_pct": float(100 * np.percentile(r, 95)),
            "aggregate_pct": float(100 * (tc.sum() / best.sum() - 1.0)), "best_picked_pct": float(100 * np.mean(r == 0))}


def _choices(X, M, theta, classes=None):
    """Network (theta) and cost-model choices for feature rows X over the classes
    valid per M, restricted to `classes` when given."""
    allowed = np.ones(gj.N_CLASSES, bool) if classes is None else np.isin(np.arange(gj.N_CLASSES), classes)
    mlp_c, cm_c = [], []
    gj.selector_set_weights(theta)
    for x, m in zip(X, M):
        ok = (m > 0) & allowed
        _, p = gj.select(x, 0 if m[0] else 1)
        mlp_c.append(int(np.argmax(np.where(ok, p, -1.0))))
    gj.selector_set_weights(None)
    for x, m in zip(X, M):
        ok = (m > 0) & allowed
        t = np.array(gj.cost_model(x, 0 if m[0] else 1))
        cm_c.append(int(np.argmin(np.where(ok, t, np.inf))))
    return np.array(mlp_c), np.array(cm_c)


def evaluate_arrays(X, M, T, theta, classes=None) -> dict:
    """Regret of the network (theta), the cost model, and a fixed choice, from
    feature and timing arrays alone (optionally over a subset of the classes)."""
    if classes is not None:
        keep = np.isin(np.arange(gj.N_CLASSES), classes)
        M = M * keep
    mlp_c, cm_c = _choices(X, M, theta, classes)
    fixed = np.array([0 if m[0] else 4 for m in M])
    rep = {"mlp": regret(T, M, mlp_c), "cost_model": regret(T, M, cm_c), "always_gftr_pgb": regret(T, M, fixed)}
    t_mlp = T[np.arange(len(T)), mlp_c].sum()
    t_cm = T[np.arange(len(T)), cm_c].sum()
    rep["mlp_vs_cost_model_pct"] = float(100 * (t_mlp / t_cm - 1.0))
    rep["n"] = int(len(X))
    return rep


def evaluate(ws, X, M, T, theta, classes=None) -> dict:
    rep = evaluate_arrays(X, M, T, theta, classes)
    if classes is not None:
        M = M * np.isin(np.arange(gj.N_CLASSES), classes)
    he_c = np.array([heuristic_choice(w) for w in ws])
    he_c = np.array([c if M[i, c] > 0 else (0 if M[i, 0] else 3) for i, c in enumerate(he_c)])
    rep["paper_heuristics"] = regret(T, M, he_c)
    return rep


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


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default="selector_out")
    ap.add_argument("--data", default=None, help="reuse timings from this .npz (no re-timing)")
    ap.add_argument("--part", type=int, default=None)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--merge", default=None, metavar="DIR", help="merge the timed parts found in DIR")
    ap.add_argument("--large", default="0,0", metavar="TRAIN,TEST",
                    help="extension sets of group-bys at 2^26-2^28 rows (sample_large), appended to the main sets")
    ap.add_argument("--large-only", action="store_true", help="with --part: time only the extension sets")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    n_ltr, n_lte = (int(x) for x in args.large.split(","))
    ltr, lte = sample_large(n_ltr, 3), sample_large(n_lte, 4)
    tr, te = sample(args.train, 1), sample(args.test, 2)
    keys = ("Xtr", "Htr", "Mtr", "Ttr", "Xte", "Hte", "Mte", "Tte")
    if args.part is not None:
        src_tr, src_te, tag = (ltr, lte, "large_part") if args.large_only else (tr, te, "part")
        a, b = part_slice(len(src_tr), args.part, args.parts), part_slice(len(src_te), args.part, args.parts)
        print(f"[selector] {tag} {args.part}/{args.parts}: train {a.start}..{a.stop}, test {b.start}..{b.stop}",
              flush=True)
        arrs = build(src_tr[a]) + build(src_te[b])
        np.savez(os.path.join(args.out, f"selector_{tag}{args.part:03d}of{args.parts:03d}.npz"),
                 **dict(zip(keys, arrs)))
        return 0
    if args.merge:
        # the main parts, then (if asked for) the extension's parts
        names = [f"selector_part{i:03d}of{args.parts:03d}.npz" for i in range(args.parts)]
        if n_ltr or n_lte:
            names += [f for f in sorted(os.listdir(args.merge)) if f.startswith("selector_large_part")]
        z = [np.load(os.path.join(args.merge, f)) for f in names]
        data = {k: np.concatenate([q[k] for q in z if q[k].size]) for k in keys}
        np.savez(os.path.join(args.out, "selector_data.npz"), **data)
    elif args.data:
        data = load_data(args.data)
    else:
        data = dict(zip(keys, build(tr + ltr) + build(te + lte)))
        np.savez(os.path.join(args.out, "selector_data.npz"), **data)
    tr, te = tr + ltr, te + lte
    assert len(tr) == len(data["Xtr"]) and len(te) == len(data["Xte"]), "timed sets and samples differ"
    # train on both feature views: what the library computes alone, and with the
    # caller's hints of match ratio and skew
    Xall = np.concatenate([data["Xtr"], data["Htr"]])
    theta = train(Xall, np.concatenate([data["Mtr"]] * 2), np.concatenate([data["Ttr"]] * 2), steps=args.steps)
    theta.astype("<f4").tofile(os.path.join(args.out, "selector_weights.f32"))
    rep = {}
    for name, X in (("product_path", "X"), ("with_hints", "H")):
        rep[name] = {"train": evaluate(tr, data[X + "tr"], data["Mtr"], data["Ttr"], theta),
                     "test": evaluate(te, data[X + "te"], data["Mte"], data["Tte"], theta),
                     "test_five_classes": evaluate(te, data[X + "te"], data["Mte"], data["Tte"], theta,
                                                   classes=[0, 1, 2, 3, 4])}
    with open(os.path.join(args.out, "selector_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps(rep), flush=True)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    sys.exit(main())
