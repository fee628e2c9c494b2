import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The loaded HIP library; GPU tests fail (not skip) when it is missing."""
    from paper_2412_13547_amd import api
    return api.lib()
