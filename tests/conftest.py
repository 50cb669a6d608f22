import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only check")


@pytest.fixture(scope="session")
def golden():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def coeffs16():
    """Proposed-solver coefficients (C^E, C^B), M = 16, dt = dx1/2, from the
    oracle's App. B fit (printed weight, n = 10, w_k1 = 0.4)."""
    from oracle import stencil
    return stencil.fit_pair(16, 0.5)


@pytest.fixture(scope="session")
def coeffs16_quarter():
    """Proposed-solver coefficients (C^E, C^B), M = 16, dt = dx1/4 (the
    paper's Sec. 4.1 ratio), where C^B is a wide Ampere stencil."""
    from oracle import stencil
    return stencil.fit_pair(16, 0.25)
