import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running test")


def flush_print(*args):
    print(*args, flush=True)


@pytest.fixture(autouse=True)
def _name_the_case(request):
    # Name every GPU case before it runs so that a crash report identifies it.
    if request.node.get_closest_marker("gpu") is not None:
        flush_print(f"\n[case] {request.node.nodeid}")
    yield
