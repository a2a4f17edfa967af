import json
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def golden_instance(g):
    """SimpleNamespace instance from a golden fixture's "instance" entry."""
    d = dict(g["instance"])
    d["v"] = np.asarray(d["v"], dtype=np.float32)
    d["ore"] = np.asarray(d["ore"], dtype=np.uint8)
    d["ton"] = np.asarray(d["ton"], dtype=np.float64)
    return SimpleNamespace(**d)


@pytest.fixture(scope="session")
def tiny():
    import mpsgen
    return mpsgen.tiny_plain()
