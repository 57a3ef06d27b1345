import os
import sys

# small dense linear algebra in the pins: one BLAS thread avoids oversubscription
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _seed_torch():
    """Every test starts from the same torch generator state (CPU and GPU), so
    tests that draw with torch.randn are reproducible."""
    import torch
    torch.manual_seed(20170706)
    yield
