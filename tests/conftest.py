import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: full-size host checks (opt in with DAMN_SLOW=1)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("DAMN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="full-size host check; set DAMN_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)
