import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def golden_path(name: str) -> str:
    return os.path.join(ROOT, "tests", "golden", name)


def read_closed_forms() -> dict:
    out = {}
    with open(golden_path("closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=")
            out[k.strip()] = float(v)
    return out


@pytest.fixture(scope="session")
def closed_forms():
    return read_closed_forms()
