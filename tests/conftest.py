import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


import pytest  # noqa: E402


@pytest.fixture(params=["default", "morton"])
def morton(request):
    """Runs a test under the library's default pull-table policy and under
    one that gives every block and level all the Morton directions they
    qualify for (small meshes otherwise keep the code path only)."""
    import paper_1601_06984_amd as M
    if request.param == "morton":
        M.set_morton_policy(0.0, 1)
    try:
        yield request.param
    finally:
        M.set_morton_policy()
