import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_rows(name):
    """Numeric rows of a golden fixture (lines starting with '#' skipped)."""
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def load_matrix(name, dtype=np.float64):
    return np.array([[float(x) for x in r] for r in load_rows(name)], dtype=dtype)


def load_keyed(name):
    return {r[0]: [int(x) for x in r[1:]] for r in load_rows(name)}


@pytest.fixture
def golden():
    return GOLDEN
