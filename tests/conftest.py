import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "fullscale: multi-minute full-size case, opt-in via WEDGE_FULLSCALE=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("WEDGE_FULLSCALE") == "1":
        return
    skip = pytest.mark.skip(reason="full-size case: set WEDGE_FULLSCALE=1 to run it")
    for it in items:
        if "fullscale" in it.keywords:
            it.add_marker(skip)
