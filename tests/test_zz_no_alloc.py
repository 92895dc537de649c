"""GPU parity of gj_partition_noalloc (the partition primitive of Section 2.3
with its scratch in a static device array) against gj_partition, element by
element, on consecutive calls that reuse the array: a large input, then a
smaller one with other digit bits, then an empty one."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _both(keys, cols, bit_lo, bits, mode):
    import torch
    import paper_2312_00720_amd as gj
    from gpu_util import dev, host, say
    say(f"noalloc partition n={len(keys)} dtype={keys.dtype} bits=[{bit_lo},{bit_lo + bits}) mode={mode}")
    k, c = dev(keys), [dev(x) for x in cols]
    ref = gj.partition(k, c, bit_lo=bit_lo, bits=bits, passes=1, mode=mode, rowid=True)
    torch.cuda.synchronize()
    ok = torch.full_like(k, -7)
    oc = [torch.full_like(x, -7) for x in c]
    orow = torch.full((len(keys),), -7, dtype=torch.int32, device="cuda")
    off = torch.full(((1 << bits) + 1,), -7, dtype=torch.int32, device="cuda")
    before = torch.cuda.memory_allocated()
    gj.partition_noalloc(k, c, ok, oc, off, bit_lo=bit_lo, bits=bits, mode=mode, out_rowid=orow)
    assert torch.cuda.memory_allocated() == before
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(ok), host(ref[0]))
    for a, b in zip(oc, ref[1]):
        np.testing.assert_array_equal(host(a), host(b))
    np.testing.assert_array_equal(host(orow), host(ref[2]))
    np.testing.assert_array_equal(host(off), host(ref[3]))


def test_noalloc_partition_matches_allocating_call_twice():
    g = datagen.rng(4242)
    n1 = (1 << 24) + 777  # several 16384-row tiles per chunk, ragged tail
    keys = datagen.raw_keys(n1, seed=11)
    cols = [g.integers(-2**31, 2**31, size=n1, dtype=np.int64).astype(np.int32),
            g.integers(-2**62, 2**62, size=n1, dtype=np.int64)]
    _both(keys, cols, 3, 8, "bits")
    n2 = 70001  # smaller, fewer digits: the array keeps the first call's contents
    keys2 = datagen.raw_keys(n2, seed=12, key_bytes=8)
    cols2 = [g.integers(-2**31, 2**31, size=n2, dtype=np.int64).astype(np.int32)]
    _both(keys2, cols2, 40, 5, "hash")
    _both(np.zeros(0, np.int32), [], 0, 4, "ordered")


def test_noalloc_partition_rejects_two_pass_requests():
    import torch
    import paper_2312_00720_amd as gj
    k = torch.arange(1000, dtype=torch.int32, device="cuda")
    off = torch.empty((1 << 9) + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(gj.GJError) as e:
        gj.partition_noalloc(k, [], torch.empty_like(k), [], off, bits=9)
    assert e.value.code == -1
