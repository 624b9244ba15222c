import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture
def say(capsys):
    """Print a progress line as it happens, past pytest's output capture
    (long oracle runs on full-size inputs would otherwise look silent)."""
    import time
    t0 = time.time()

    def _say(msg):
        with capsys.disabled():
            print(f"[{time.time() - t0:7.1f} s] {msg}", flush=True)
    return _say
