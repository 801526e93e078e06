import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: takes more than ~20 s on the CPU")


@pytest.fixture(params=["two_pass", "read_once"])
def both_schemes(request, monkeypatch):
    """Run a single-instance test under both iteration schemes (the panel
    read twice per iteration, or once with per-workgroup partials of
    P^T v): every DualSolver the test creates gets the scheme unless the
    test names one itself."""
    from paper_2406_13191_amd import _abi
    orig = _abi.make_opts

    def make_opts(*args, **kw):
        kw.setdefault("scheme", request.param)
        return orig(*args, **kw)

    monkeypatch.setattr(_abi, "make_opts", make_opts)
    return request.param
