"""The allocation-free sort entry point (gs_sort_pairs_static, scratch in
the library's static device array) against the workspace entry point
(gs_sort_pairs) on the same inputs, through the C ABI: two calls in a row,
the second smaller (its scratch still holds the first call's contents), and
both against a stable sort on the host.  Bar: bit-exact keys and values."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_static_scratch_sort_equals_workspace_sort():
    need_gpu()
    import paper_2407_00435_amd as g
    rng = np.random.default_rng(12)
    # 32-bit keys sort in 4 passes (result in place), 18-bit keys in 3
    # (result copied back from the second buffers)
    for n, bits in ((3_000_001, 32), (123_457, 18)):
        say(f"static-scratch sort: n {n}, bits {bits}")
        keys = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
        vals = rng.permutation(n).astype(np.uint32)
        ka = torch.from_numpy(keys.view(np.int32).copy()).cuda()
        va = torch.from_numpy(vals.view(np.int32).copy()).cuda()
        kb, vb = ka.clone(), va.clone()
        g.gs_sort_pairs(ka, va, bits)
        g.gs_sort_pairs_static(kb, vb, bits)
        torch.cuda.synchronize()
        assert torch.equal(ka, kb) and torch.equal(va, vb)
        order = np.argsort(keys, kind="stable")
        np.testing.assert_array_equal(kb.cpu().numpy().view(np.uint32), keys[order])
        np.testing.assert_array_equal(vb.cpu().numpy().view(np.uint32), vals[order])
    # beyond the static scratch: refused on the host before anything runs
    L = g.lib()
    assert L.gs_sort_pairs_static(None, None, None, None, g.binding.SORT_STATIC_MAX_KEYS + 1, 32,
                                  None) == g.binding.GS_ERR_CAPACITY
    assert b"maximum" in g.binding.raw_lib().gs_last_error()
