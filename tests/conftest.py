import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle's passes are OpenMP loops that take every core by default; under
# pytest-xdist each worker would start that many threads and the CPUs would be
# oversubscribed many times over. Workers share the cores out instead (read by
# the OpenMP runtime when the oracle library is first loaded).
if os.environ.get("PYTEST_XDIST_WORKER") and "OMP_NUM_THREADS" not in os.environ:
    _workers = max(1, int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1")))
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // _workers))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C-ABI)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.load()
    return O


@pytest.fixture(scope="session")
def gpu():
    """The GPU binding; fails loudly when the HIP library or the GPU is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test collected on a machine without a GPU")
    import paper_1606_09432_amd as lb
    lb.load_library()
    return lb
