import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through libsx on cuda:0)")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


@pytest.fixture(scope="session")
def sxctx():
    """One libsx context for the whole GPU session."""
    from paper_0912_4273_amd import sx
    ctx = sx.Context(device=0)
    yield ctx
    ctx.close()
