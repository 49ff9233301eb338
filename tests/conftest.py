import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly when the
    built extension is missing."""
    import paper_1307_0491_amd as sve
    sve.require_device()
    return sve


def pytest_runtest_setup(item):
    try:
        import gpu_helpers
    except ImportError:
        return
    gpu_helpers.CURRENT_TEST = item.nodeid


def pytest_sessionfinish(session, exitstatus):
    """With SVE_PARITY_REPORT set, write every field comparison of the GPU
    tests (relative errors per field, the transverse momentum also against
    its own maximum) to that file as JSON."""
    path = os.environ.get("SVE_PARITY_REPORT")
    if not path:
        return
    try:
        import gpu_helpers
    except ImportError:
        return
    import json
    with open(path, "w") as f:
        json.dump(gpu_helpers.RECORDS, f)
