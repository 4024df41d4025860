import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def pytest_runtest_logreport(report):
    """Print a failure as soon as it happens, so that a later crash of the
    process cannot hide it."""
    if report.failed:
        import sys as _sys
        _sys.stderr.write(f"\n[failed] {report.nodeid} ({report.when})\n{report.longreprtext}\n")
        _sys.stderr.flush()
