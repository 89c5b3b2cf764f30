import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # the tests check the in-tree library; another build selected through the
    # binding's STARK_LIBRARY variable would be tested in its place
    if os.environ.get("STARK_LIBRARY"):
        raise pytest.UsageError("STARK_LIBRARY is set: the tests run the in-tree libstark.so only; unset it")
