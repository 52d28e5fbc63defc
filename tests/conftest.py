import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist the workers share the host's cores: cap the oracle's
# OpenMP threads per worker and let idle threads sleep instead of spinning
# (oversubscribed spinning threads slow the oracle runs many times over).
_WORKERS = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1"))
if _WORKERS > 1:
    os.environ.setdefault("ORACLE_MAX_THREADS", str(max(1, (os.cpu_count() or 1) // _WORKERS)))
    os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU runs")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
