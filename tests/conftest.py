import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    """Rows of a '|'-separated golden file; '#' lines are comments.

    Matrix fields use ';' between rows and spaces between entries.
    """
    import numpy as np

    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            fields = [x.strip() for x in line.split("|")]
            out = [fields[0]]
            for fld in fields[1:]:
                mat = [[float(v) for v in r.split()] for r in fld.split(";")]
                out.append(np.array(mat, dtype=np.float64))
            rows.append(out)
    return rows


@pytest.fixture
def golden():
    return read_golden
