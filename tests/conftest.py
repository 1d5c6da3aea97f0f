import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (still part of the default run)")


def _cores():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


@pytest.fixture(scope="session")
def oracle():
    """The C oracle, using up to 16 host threads."""
    from oracle import ref
    o = ref.default()
    o.set_threads(min(16, _cores()))
    return o


@pytest.fixture(scope="session")
def oracle1():
    """The C oracle pinned to one thread (for timing-independent small runs)."""
    from oracle import ref
    return ref.Oracle()
