import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_golden(name):
    """Parse a golden fixture with [section] headers and whitespace-separated rows."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = []
                continue
            out[cur].append([float(t) for t in line.split()])
    import numpy as np
    return {k: np.array(v) for k, v in out.items()}


@pytest.fixture
def golden():
    return load_golden
