"""Pins for the group-count sketch oracle: HyperLogLog (Flajolet, Fusy,
Gandouet and Meunier, 2007) over the MurmurHash3 finalizer of the keys, and the
count of key bytes that vary.

The registers are pinned by what the sketch's definition fixes (a register per
top-bits value, the largest first-one position of the remaining bits; the
union of two key sets is the register-wise max; repeating keys changes
nothing), the estimate by its published standard error (1.04 / sqrt(m)) on
known cardinalities, and by linear counting's exactness on tiny sets.
"""
import numpy as np
import pytest

import oracle

BITS = 10
M = 1 << BITS


def distinct_keys(g, seed, key_bytes=4):
    rng = np.random.default_rng(seed)
    if key_bytes == 4:
        k = rng.choice(np.int64(1) << 32, size=g, replace=False) - (1 << 31)
        return k.astype(np.int32)
    k = rng.integers(-(1 << 63), (1 << 63) - 1, size=g, dtype=np.int64)
    return np.unique(k)


def test_single_key_register():
    # one key: exactly its register is set, to the first-one position read off
    # the hash's bit string (the hash itself is pinned to published vectors)
    for key in (1, -1, 12345, 2**31 - 1, -(2**31)):
        h = oracle.digit_source(key, 4, oracle.DIGIT_HASH)
        regs = oracle.hll_registers(np.array([key], np.int32), BITS)
        rest = format(h & ((1 << (32 - BITS)) - 1), f"0{32 - BITS}b")
        rho = rest.index("1") + 1 if "1" in rest else 32 - BITS + 1
        expect = np.zeros(M, np.uint32)
        expect[h >> (32 - BITS)] = rho
        np.testing.assert_array_equal(regs, expect)


def test_zero_hash_has_the_largest_rank():
    # key 0 hashes to 0 (pinned vector): all remaining bits are zero
    regs = oracle.hll_registers(np.array([0], np.int32), BITS)
    assert regs[0] == 32 - BITS + 1 and np.count_nonzero(regs) == 1


def test_union_is_registerwise_max():
    a, b = distinct_keys(5000, 1), distinct_keys(7000, 2)
    ra, rb = oracle.hll_registers(a, BITS), oracle.hll_registers(b, BITS)
    rab = oracle.hll_registers(np.concatenate([a, b]), BITS)
    np.testing.assert_array_equal(rab, np.maximum(ra, rb))


def test_duplicates_change_nothing():
    k = distinct_keys(3000, 3)
    rng = np.random.default_rng(4)
    rep = rng.permutation(np.repeat(k, rng.integers(1, 6, size=len(k))))
    np.testing.assert_array_equal(oracle.hll_registers(rep, BITS), oracle.hll_registers(k, BITS))
    assert oracle.hll_estimate(rep) == pytest.approx(oracle.hll_estimate(k), rel=0, abs=0)


@pytest.mark.parametrize("key_bytes", [4, 8])
@pytest.mark.parametrize("g", [1000, 10_000, 100_000, 1_000_000])
def test_estimate_within_published_error(g, key_bytes):
    # standard error 1.04 / sqrt(m) = 3.25% at m = 1024; allow four of them
    est = oracle.hll_estimate(distinct_keys(g, 10 + g % 97, key_bytes))
    assert abs(est / g - 1.0) < 4 * 1.04 / np.sqrt(M)


def test_small_sets_use_linear_counting():
    # well below 5m/2 the estimate is linear counting over the zero registers,
    # and 200 keys leave most registers zero
    k = distinct_keys(200, 5)
    regs = oracle.hll_registers(k, BITS)
    zeros = int(np.count_nonzero(regs == 0))
    assert oracle.hll_estimate(k) == pytest.approx(M * np.log(M / zeros), rel=1e-12)
    assert abs(oracle.hll_estimate(k) / 200 - 1.0) < 0.05


def test_estimate_capped_and_empty():
    assert oracle.hll_estimate(np.array([7], np.int32)) == 1.0
    assert oracle.hll_estimate(np.array([], np.int32)) == 0.0


def test_varying_key_bytes_brute_force():
    rng = np.random.default_rng(6)
    cases = [np.array([5, 5, 5], np.int32), np.array([0, 255], np.int32), np.array([0, 256], np.int32),
             np.array([-1, 0], np.int32), rng.integers(0, 1 << 20, 50).astype(np.int32),
             rng.integers(-(1 << 40), 1 << 40, 50).astype(np.int64), np.array([], np.int64)]
    for k in cases:
        kb = k.dtype.itemsize
        brute = sum(1 for b in range(kb)
                    if len({(int(x) % (1 << (8 * kb))) >> (8 * b) & 0xFF for x in k.tolist()}) > 1)
        assert oracle.varying_key_bytes(k) == brute
