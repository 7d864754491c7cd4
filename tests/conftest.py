import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on the device)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _device_first(request):
    """When GPU tests run, bring up the device (torch's runtime and the
    library's) before any test builds its inputs on the host."""
    if not any(item.get_closest_marker("gpu") for item in request.session.items):
        yield
        return
    import torch
    if torch.cuda.is_available():
        from paper_1404_0447_amd import selinv as S
        from paper_1404_0447_amd import workloads as W
        S.Plan.from_matrix(W.laplacian((4, 4), shift=0.1)).bind()
        torch.cuda.synchronize()
    yield
