import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer checks (statistical CPU checks, full-size GPU runs)")


_torch_cuda_ready = False


@pytest.fixture(autouse=True)
def _torch_runtime_before_library(request):
    """GPU tests: bring up torch's HIP runtime before the first test runs, so that its
    initialisation does not depend on which library calls (and host work) came earlier
    in the session."""
    global _torch_cuda_ready
    if not _torch_cuda_ready and request.node.get_closest_marker("gpu") is not None:
        _torch_cuda_ready = True
        try:
            import torch
        except ImportError:
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
    yield
