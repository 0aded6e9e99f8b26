import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libtpf.so")
    config.addinivalue_line("markers", "slow: long-running case")


@pytest.fixture(scope="session")
def gpu():
    """The CUDA/HIP torch device; GPU tests fail loudly if the library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this container")
    import paper_2403_04578_amd as tpf
    tpf.load_library()  # raises ImportError when libtpf.so was not built
    return torch.device("cuda:0")
