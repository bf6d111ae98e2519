import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    import oracle as O
    O.build(force=False)
    return O


# Measured errors of the GPU results against the oracle, by name; written as
# JSON to the path in VTX_ERROR_REPORT when the session ends.
_ERRORS = {}


@pytest.fixture(scope="session")
def errlog():
    def record(name, value):
        _ERRORS[name] = float(value)
    return record


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("VTX_ERROR_REPORT")
    if path and _ERRORS:
        with open(path, "w") as f:
            json.dump(_ERRORS, f, indent=1, sort_keys=True)
