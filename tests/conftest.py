import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.load()
    return oracle


@pytest.fixture(params=["flat", "persistent"])
def form(request, monkeypatch):
    """The batched call's two forms (SS_BATCH_FORM); outputs must not depend on it."""
    if request.param == "persistent":
        monkeypatch.setenv("SS_BATCH_FORM", "persistent")
    else:
        monkeypatch.delenv("SS_BATCH_FORM", raising=False)
    return request.param
