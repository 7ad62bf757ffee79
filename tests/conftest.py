import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# GPU files in the order they are run: stage parity against the oracle first,
# then the composed paths, the full sizes and the GPU-against-GPU comparisons,
# so that a failure late in the list (under -x) hides as few oracle checks as
# possible.  Files not listed keep their place after these (the allocation-free
# entry point's test, test_zz_*, is collected last by name).
GPU_ORDER = ("test_gpu_parity.py", "test_gpu_edge.py", "test_gpu_sort.py", "test_gpu_prune.py", "test_gpu_loss.py",
             "test_gpu_queue.py", "test_gpu_merge.py", "test_gpu_streamed.py", "test_gpu_fr_bwd.py", "test_gpu_ctx.py",
             "test_gpu_hvsq.py", "test_gpu_batched_oracle.py", "test_gpu_batched.py",
             "test_gpu_fullsize.py")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")


def pytest_collection_modifyitems(session, config, items):
    def rank(item):
        name = os.path.basename(str(item.fspath))
        if name in GPU_ORDER:
            return (1, GPU_ORDER.index(name))
        if name.startswith("test_zz_"):
            return (3, 0)
        if name.startswith("test_gpu_"):
            return (2, 0)
        return (0, 0)
    items.sort(key=rank)  # stable: keeps the order inside each file


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
