import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def _flush_name(item):
    # name the case before it runs, so a GPU failure that ends the process
    # still leaves the test's name in the log
    sys.stdout.write("\n[case] %s\n" % item.nodeid)
    sys.stdout.flush()


@pytest.hookimpl(tryfirst=True)
def pytest_runtest_setup(item):
    if item.get_closest_marker("gpu") is not None:
        _flush_name(item)
