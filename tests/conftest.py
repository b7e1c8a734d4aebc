import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_golden(name):
    """Lines of a golden fixture with comments and blanks removed."""
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.lstrip().startswith("#")]


@pytest.fixture
def golden():
    return read_golden


@pytest.fixture(scope="session")
def c0_inputs():
    import synth
    return synth.synth_image(64, 64, 42), synth.xavier_mlp((12, 32, 32, 15), 7)
