import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_table(name):
    """Parse a golden residual-history table: {column: [values or None]}."""
    cols = ["n", "F64", "F32", "F16", "IR32-16", "IR-GM"]
    out = {c: [] for c in cols}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            for c, p in zip(cols, parts):
                out[c].append(None if p == "-" else float(p))
    return out


@pytest.fixture(scope="session")
def table2():
    return load_table("table2_heq_n4096_c0.99.txt")


@pytest.fixture(scope="session")
def table3():
    return load_table("table3_heq_n4096_c0.9999.txt")
