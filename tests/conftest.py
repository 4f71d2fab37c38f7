import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _read_enum_golden():
    """tests/golden/enum_pairs.txt: B intervals, then per query (start, end,
    expected set of B indices, expected backward-scan order)."""
    B, Q = [], []
    with open(os.path.join(ROOT, "tests", "golden", "enum_pairs.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line.startswith("B"):
                _, s, e = line.split()
                B.append((int(s), int(e)))
            else:
                head, st, sc = line.split(";")
                _, s, e = head.split()
                Q.append((int(s), int(e), [int(v) for v in st.split()], [int(v) for v in sc.split()]))
    return B, Q


@pytest.fixture
def enum_golden():
    return _read_enum_golden()
