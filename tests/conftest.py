import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU case, run with MB_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("MB_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="long CPU case; set MB_SLOW=1 to run")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as O
    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        O.build()
    yield


@pytest.fixture(autouse=True)
def _release_device_memory():
    """Frees the device memory a test leaves behind (a failing full-size test
    would otherwise hold its buffers while the next one allocates)."""
    yield
    import gc
    gc.collect()
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.empty_cache()
    except ImportError:
        pass
