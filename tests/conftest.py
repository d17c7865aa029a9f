import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU-side inputs (oracle at scale)")


@pytest.fixture(scope="session", autouse=True)
def _built_host_libs():
    """Build the CPU-side helper libraries only when they are missing."""
    import oracle
    import synth

    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build(force=False)
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=False)
    yield
