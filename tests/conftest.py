import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle._load()
    return oracle


@pytest.fixture(autouse=True)
def _live_progress(request):
    """Let gpu_helpers.say print past pytest's output capture."""
    try:
        import gpu_helpers
    except ImportError:
        yield
        return
    gpu_helpers.CAPMAN = request.config.pluginmanager.getplugin("capturemanager")
    yield
