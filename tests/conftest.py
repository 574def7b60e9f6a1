import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


_CACHE = {}


def workload(name, **kw):
    """Process-wide cache of synthetic workloads (they take seconds to build)."""
    from workloads import configs
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = configs.BUILDERS[name](**kw)
    return _CACHE[key]


@pytest.fixture(scope="session")
def tiny():
    return workload("tiny")


@pytest.fixture(autouse=True)
def _release_cached_device_memory():
    """After each test, hand the memory torch's caching allocator keeps back to the device:
    the library allocates its own buffers with hipMalloc, outside that cache."""
    yield
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        gc.collect()
        torch.cuda.empty_cache()
