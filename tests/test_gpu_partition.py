"""GPU parity: the radix-partition primitive (Section 2.3) against the oracle's
stable sort by digit, element by element."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def _run(keys, cols, bit_lo, bits, passes, mode, rowid=True):
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    say(f"partition n={len(keys)} dtype={keys.dtype} bits=[{bit_lo},{bit_lo + bits}) "
        f"passes={passes} mode={mode} cols={len(cols)}")
    k, c, r, off = gj.partition(dev(keys), [dev(x) for x in cols], bit_lo=bit_lo, bits=bits,
                                passes=passes, mode=mode, rowid=rowid)
    return host(k), [host(x) for x in c], (host(r) if rowid else None), host(off)


CASES = [
    # n, key_bytes, bit_lo, bits, passes, mode
    (0, 4, 0, 4, 1, "bits"),
    (1, 4, 0, 8, 1, "bits"),
    (1000, 4, 0, 3, 1, "bits"),
    (4097, 4, 2, 8, 1, "bits"),          # one full tile plus one row
    (70001, 4, 0, 16, 2, "bits"),        # several chunks, ragged tail, two passes
    (70001, 4, 5, 11, 2, "hash"),
    (50000, 4, 24, 8, 1, "ordered"),
    (50000, 8, 0, 12, 2, "bits"),
    (50000, 8, 40, 9, 2, "hash"),
    (300000, 4, 0, 13, 2, "bits"),       # multiple tiles per chunk
]


@pytest.mark.parametrize("case", CASES)
def test_partition_matches_oracle(case):
    n, kb, lo, bits, passes, mode = case
    g = datagen.rng(n + bits)
    keys = datagen.raw_keys(n, seed=n + lo, key_bytes=kb)
    cols = [g.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32),
            g.integers(-2**62, 2**62, size=n, dtype=np.int64)]
    k, c, r, off = _run(keys, cols, lo, bits, passes, mode)
    perm, hist = oracle.partition(keys, lo, bits, getattr(oracle, "DIGIT_" + mode.upper()))
    np.testing.assert_array_equal(k, keys[perm])
    np.testing.assert_array_equal(c[0], cols[0][perm])
    np.testing.assert_array_equal(c[1], cols[1][perm])
    np.testing.assert_array_equal(r, perm.astype(np.int32))
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(hist)]).astype(np.int32))


@pytest.mark.timeout(600)
def test_partition_chunks_of_several_tiles():
    """Past 4096 tiles, a chunk spans several 16384-row tiles: the scatter's
    next-tile prefetch and the partial last tile of every segment are used."""
    n = (1 << 26) + 12345
    g = datagen.rng(77)
    keys = datagen.raw_keys(n, seed=78)
    cols = [g.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)]
    k, c, r, off = _run(keys, cols, 0, 16, 2, "bits")
    perm, hist = oracle.partition(keys, 0, 16, oracle.DIGIT_BITS)
    np.testing.assert_array_equal(r, perm.astype(np.int32))
    np.testing.assert_array_equal(k, keys[perm])
    np.testing.assert_array_equal(c[0], cols[0][perm])
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(hist)]).astype(np.int32))


def test_partition_skewed_digits():
    """A single hot digit (all keys equal) and Zipf-skewed keys stay stable."""
    n = 200000
    keys = np.full(n, 12345, np.int32)
    vals = np.arange(n, dtype=np.int32)
    k, c, r, off = _run(keys, [vals], 0, 10, 2, "bits")
    np.testing.assert_array_equal(c[0], vals)
    d = datagen.groupby_input(n, 1 << 12, 1, seed=3, alpha=1.2)
    k, c, r, off = _run(d["key"], d["vals"], 0, 12, 2, "hash")
    perm, hist = oracle.partition(d["key"], 0, 12, oracle.DIGIT_HASH)
    np.testing.assert_array_equal(r, perm.astype(np.int32))
    np.testing.assert_array_equal(c[0], d["vals"][0][perm])


def test_partition_is_deterministic():
    keys = datagen.raw_keys(123457, seed=8)
    a = _run(keys, [], 0, 14, 2, "bits")
    b = _run(keys, [], 0, 14, 2, "bits")
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])
