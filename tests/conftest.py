import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session", params=["default", "plain"])
def oracle_any(request):
    """The oracle's functions bound to its default build (rounding order fixed
    by its stated readings) or to its plain build (textbook order, the C
    library's sin/cos/exp): pins that hold for any rounding order run on both."""
    from oracle import oracle as O
    v = O.View(plain=request.param == "plain")
    v.lib()
    return v
