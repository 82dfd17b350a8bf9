import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libsil.so")


@pytest.fixture(scope="session", autouse=True)
def _built_host_libs():
    """Build the oracle and the input generator (plain C, seconds) if absent."""
    from oracle import build as ob
    from synth import synth as sy
    if not os.path.exists(ob.LIB):
        ob.build()
    if not os.path.exists(sy.LIB):
        sy.build()
