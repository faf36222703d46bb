import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libgrpic.so")


def load_tab_paths():
    """Rows of Table tab:paths from tests/golden/tab_paths.txt."""
    rows = {}
    with open(os.path.join(ROOT, "tests", "golden", "tab_paths.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            f = line.split()
            th = f[7]                     # "pi/2" or "pi/2-0.1"
            assert th.startswith("pi/2")
            theta = math.pi / 2 + (float(th[4:]) if len(th) > 4 else 0.0)
            rows[f[0]] = dict(a=float(f[1]), Bz=float(f[2]), u=(float(f[3]), float(f[4]), float(f[5])),
                              r=float(f[6]), theta=theta)
    return rows


@pytest.fixture(scope="session")
def tab_paths():
    return load_tab_paths()
