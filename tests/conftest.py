import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The library keeps compiled kernels and the autotuner's stored launch shapes
# in its cache directory, and a submission without a tuning uses a stored
# shape.  A fresh directory per test session makes "no tuning" mean the
# library's defaults, whatever ran before on this machine.
os.environ["CWC_CACHE_DIR"] = tempfile.mkdtemp(prefix="cwc-test-cache-")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
