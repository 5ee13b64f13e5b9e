import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle.lib()


def _flush_print(msg):
    print(msg, flush=True)


@pytest.fixture(autouse=True)
def _announce(request):
    # Name the case before it runs, so a GPU fault can be attributed.
    if request.node.get_closest_marker("gpu") is not None:
        _flush_print(f"\n[gpu-case] {request.node.nodeid}")
    yield
