import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# The oracle's library FFTs may use the host's cores (its arithmetic is unchanged).
try:
    _ncpu = len(os.sched_getaffinity(0))
except AttributeError:
    _ncpu = os.cpu_count() or 1
os.environ.setdefault("ORACLE_FFT_WORKERS", str(max(1, min(16, _ncpu))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def lib():
    """The GPU library binding; skips when no GPU is visible."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1812_07357_amd import psatd

    return psatd
