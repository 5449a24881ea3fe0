import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_cpu_libs():
    """Build the oracle and the input generator if no build is present (gcc only)."""
    from oracle import build as obuild
    if not os.path.exists(obuild.LIB):
        obuild.build()
    from paper_1911_02696_amd import build as pbuild
    if not os.path.exists(pbuild.GEN_LIB):
        pbuild.build_gen()


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.get()
