import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: full-size CPU checks (minutes); run with DDF_RUN_SLOW=1")


def pytest_collection_modifyitems(config, items):
    # the full-size table checks take minutes: only on request
    if os.environ.get("DDF_RUN_SLOW"):
        return
    import pytest
    skip = pytest.mark.skip(reason="full-size check: set DDF_RUN_SLOW=1")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
