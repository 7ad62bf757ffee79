"""The radix sort used for the depth and tile passes (Section 2.1 "Sorting"):
bit-exact against numpy's stable sort for every partition size, with
ragged sizes (not multiples of a partition) and the digit widths the tile
keys use (9 bits: one pass of 512 digits with 8192-key partitions)."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("part", [4096, 8192, 16384])
@pytest.mark.parametrize("bits,n", [(7, 1000), (9, 500_001), (9, 8192), (14, 333_333), (18, 1_234_567),
                                    (32, 777_777), (32, 1)])
def test_sort_pairs_bit_exact(part, bits, n):
    need_gpu()
    import paper_2407_00435_amd as g
    say("sort", part, bits, n)
    g.gs_set_tuning("radix_part", part)
    rng = np.random.default_rng(bits * 1000 + n)
    if bits in (9, 14):
        # tile ids with heavy skew: a few tiles hold most keys
        keys = np.minimum(rng.zipf(1.3, n), (1 << bits) - 1).astype(np.uint32)
    else:
        keys = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    g.gs_sort_pairs(kt, vt, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint32), keys[order])
    np.testing.assert_array_equal(vt.cpu().numpy().view(np.uint32), vals[order])
    g.gs_set_tuning("radix_part", 8192)


@pytest.mark.parametrize("part", [4096, 8192])
@pytest.mark.parametrize("pattern", ["top", "middle_and_top", "all_equal", "bottom"])
def test_sort_pairs_constant_digits(part, pattern):
    """Keys whose 8-bit digits are the same for every key in some passes
    (every key lands in one digit of those passes) sort like any others."""
    need_gpu()
    import paper_2407_00435_amd as g
    say("sort constant digits", part, pattern)
    g.gs_set_tuning("radix_part", part)
    n = 300_007
    rng = np.random.default_rng(len(pattern) * 7 + part)
    r = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    if pattern == "top":
        keys = (r & 0x00FFFFFF) | 0x40000000
    elif pattern == "middle_and_top":
        keys = (r & 0x00FF00FF) | 0x12003400
    elif pattern == "all_equal":
        keys = np.full(n, 0x3F8000AB, dtype=np.uint32)
    else:
        keys = (r & 0xFFFFFF00) | 0x7
    keys = keys.astype(np.uint32)
    vals = rng.permutation(n).astype(np.uint32)
    kt = torch.from_numpy(keys.view(np.int32)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    g.gs_sort_pairs(kt, vt, 32)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint32), keys[order])
    np.testing.assert_array_equal(vt.cpu().numpy().view(np.uint32), vals[order])
    g.gs_set_tuning("radix_part", 8192)
