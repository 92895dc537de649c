"""The paper's analytical bandwidth models, evaluated in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

All costs are in seconds; bandwidths in bytes/second. B_G is the peak
sequential bandwidth of global memory, B_R the random-access bandwidth.

Sections followed:
  * random-access bandwidth from the clustered/unclustered gather profile
    (Section 4.1.1, Table 1);
  * sort-based group-by, GFTR vs GFUR (Section 4.1.3);
  * partitioned hash join, GFTR vs GFUR against the match ratio (Section 4.1.4);
  * dictionary encoding for sort-based group-by (Section 4.4, Table 2);
  * the group-by decision tree (Section 5.2, summary figure) and the join
    heuristics of the conclusion (Section 7).

Readings where the paper is silent or inconsistent:
  * the per-warp unique-group count u = min(W, g) uses the warp width W
    (32 on the paper's GPU); the random-access discount is capped at B_G/24;
  * the join model is applied per relation with N = that relation's rows and
    M = output rows; under GFTR the first payload column of each side moves with
    the key and costs only its clustered gather (Section 4.1.4);
  * the dictionary model picks the memory tier of the hash table by whether
    (k+4)*g bytes fit: L1 (192 KiB, 12*B_G), L2 (40 MiB, 4.5*B_G), else B_G.
    These constants reproduce the printed estimates of the dictionary-encoding
    figure; the 4-byte L2 rows of Table 2 instead imply about 3*B_G.
"""
from __future__ import annotations

import math

A100_BG = 1555e9  # bytes/s, the paper's GPU (Section 5)


def random_bw_ratio(cycles_unclustered: float = 12_052_942,
                    cycles_clustered: float = 1_414_398) -> float:
    """B_G / B_R from the gather profile (Section 4.1.1).

    Both gathers read the map and write the output sequentially (8 bytes per
    item at B_G); they differ in reading the input (4 bytes per item at B_G or
    at B_R). With s = time ratio: 8/B_G + 4/B_R = s * 12/B_G.
    """
    s = cycles_unclustered / cycles_clustered
    return (12.0 * s - 8.0) / 4.0


# ---- Section 4.1.3: sort-based group-by --------------------------------------

def sgb_sort_cost(n: float, bg: float = A100_BG) -> float:
    """C_S: histogram read plus 4 radix passes, each reading and writing a
    4-byte key and a 4-byte value: 17 x 4 bytes per row."""
    return 17.0 * n * 4.0 / bg


def sgb_permute_cost(n: float, g: float, bg: float = A100_BG, warp: int = 32,
                     rand_div: float = 24.0) -> float:
    """C_P: unclustered gather of one 4-byte column: read IDs and write results
    sequentially, read payloads at max(B_G/u, B_G/24) with u = min(warp, g)."""
    u = min(float(warp), float(g))
    bw_payload = max(bg / u, bg / rand_div)
    return 2.0 * n * 4.0 / bg + n * 4.0 / bw_payload


def sgb_ur_minus_tr(n: float, g: float, n_cols: int = 2, bg: float = A100_BG,
                    warp: int = 32) -> float:
    """Time(SGB-UR) - Time(SGB-TR) for n_cols value columns.

    UR sorts (key, id) once and permutes every column; TR sorts (key, column)
    per column, the first of which replaces UR's (key, id) sort."""
    return n_cols * sgb_permute_cost(n, g, bg, warp) - (n_cols - 1) * sgb_sort_cost(n, bg)


# ---- Section 4.1.4: partitioned hash join ----------------------------------------

def phj_gfur_col_cost(m: float, bg: float = A100_BG, rand_div: float = 24.0) -> float:
    """C_1: unclustered gather of M of N 4-byte values."""
    return 2.0 * 4.0 * m / bg + 4.0 * m / (bg / rand_div)


def phj_gftr_col_cost(n: float, m: float, bg: float = A100_BG, free: bool = False) -> float:
    """C_2: partition the column with its keys on 16 bits (histogram + 2 passes,
    each reading and writing key and value), then a clustered gather of M
    (read ID, read value, write). `free`: the column rides with the key."""
    part = 0.0 if free else (4.0 * n + 2.0 * 4.0 * 4.0 * n)
    return (part + 3.0 * 4.0 * m) / bg


def phj_ur_minus_tr(n_r: float, n_s: float, m: float, c_r: int = 2, c_s: int = 2,
                    bg: float = A100_BG) -> float:
    """Time(PHJ-UR) - Time(PHJ-TR) from the per-column models, per side."""
    diff = 0.0
    for n, c in ((n_r, c_r), (n_s, c_s)):
        ur = c * phj_gfur_col_cost(m, bg)
        tr = sum(phj_gftr_col_cost(n, m, bg, free=(j == 0)) for j in range(c))
        diff += ur - tr
    return diff


def phj_crossover_mr(extra_cols_partitioned: int = 1) -> float:
    """Match ratio above which GFTR beats GFUR for one column
    (C_1 = 104M > C_2 = 36N + 12M  <=>  mr > 36/92)."""
    return 36.0 / 92.0


# ---- Section 4.4: dictionary encoding ------------------------------------------

L1_BYTES = 192 * 1024
L2_BYTES = 40 * 1024 * 1024


def de_tier_bw(k: int, g: float, bg: float = A100_BG, l1_mult: float = 12.0,
               l2_mult: float = 4.5) -> float:
    size = (k + 4) * g
    if size <= L1_BYTES:
        return l1_mult * bg
    if size <= L2_BYTES:
        return l2_mult * bg
    return bg


def de_encode_cost(n: float, g: float, k: int, bg: float = A100_BG, **kw) -> float:
    """D(N, g): build (read g keys, write g entries at B_M/min(g,24)) plus probe
    (read N keys, write N codes, touch N entries at B_M/min(g,24))."""
    bm = de_tier_bw(k, g, bg, **kw)
    u = min(g, 24.0)
    build = k * g / bg + (k + 4) * g / (bm / u)
    probe = (k * n + 4 * n) / bg + (k + 4) * n / (bm / u)
    return build + probe


def de_c1(n: float, k: int, p: int, bg: float = A100_BG) -> float:
    """Sort p 4-byte payload columns with k-byte keys in k passes."""
    return p * (k * n + k * n * 2 * (k + 4)) / bg


def de_c2(n: float, g: float, k: int, p: int, bg: float = A100_BG, **kw) -> float:
    """Encode keys, then sort p columns on ceil(log2 g / 8) passes of 4-byte codes."""
    passes = math.ceil(math.log2(g) / 8.0) if g > 1 else 0
    return de_encode_cost(n, g, k, bg, **kw) + p * (4 * n + passes * n * 2 * (4 + 4)) / bg


def de_gain(n: float, g: float, k: int, p: int = 1, bg: float = A100_BG, **kw) -> float:
    """Time(SGB-TR) - Time(SGB-DE-TR) = C_1 - C_2."""
    return de_c1(n, k, p, bg) - de_c2(n, g, k, p, bg, **kw)


def de_min_payloads(n: float, g: float, k: int, bg: float = A100_BG, p_max: int = 64, **kw):
    """Smallest p with C_2 < C_1 (Table 2), or None."""
    for p in range(1, p_max + 1):
        if de_c2(n, g, k, p, bg, **kw) < de_c1(n, k, p, bg):
            return p
    return None


# ---- Heuristics -------------------------------------------------------------------

def groupby_decision(must_sort: bool, de_pays: bool, hgb_fits_lds: bool, high_skew: bool) -> str:
    """Group-by decision tree (Section 5.2 summary figure)."""
    if must_sort:
        return "SGB-DE-TR" if de_pays else "SGB-TR"
    if hgb_fits_lds:
        return "HGB"
    if high_skew:
        return "SGB-DE-TR" if de_pays else "SGB-TR"
    return "PGB-TR"


def join_decision(match_ratio: float, skewed_fk: bool, eight_byte: bool) -> str:
    """Join heuristic (Section 7): PHJ-TR when mr >= 25%, skewed foreign keys,
    or 8-byte keys/payloads; otherwise PHJ-UR."""
    if match_ratio >= 0.25 or skewed_fk or eight_byte:
        return "GFTR"
    return "GFUR"
