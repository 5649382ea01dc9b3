import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: paper-scale check, run with AMG_EIG_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("AMG_EIG_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="paper-scale check; set AMG_EIG_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
