import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; parity tests of the HIP path")
    config.addinivalue_line("markers", "slow: CPU tests that take more than a few seconds")


def pytest_runtest_logstart(nodeid, location):
    # name the case before any GPU step so a failing run says which one it was
    if os.environ.get("BLDTT_ANNOUNCE"):
        print(f"\n[case] {nodeid}", flush=True)
