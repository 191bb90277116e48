import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# torch bundles its own HIP runtime under the same soname as the system one
# the library links; loading torch first makes both use torch's copy.  With
# the library loaded first, a later torch import binds to the system runtime
# and reports no device.  Tests that use torch streams rely on this order.
import torch  # noqa: E402,F401


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
