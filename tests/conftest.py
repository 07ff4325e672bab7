import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def read_golden(name):
    """Parse a tests/golden fixture: '# ... shape r c' headers start a named
    matrix; other '#' lines are comments."""
    path = os.path.join(ROOT, "tests", "golden", name)
    mats, cur, key = {}, None, None
    with open(path) as f:
        for line in f:
            s = line.strip()
            if not s:
                continue
            if s.startswith("#"):
                toks = s[1:].split()
                if "shape" in toks:
                    i = toks.index("shape")
                    key = " ".join(toks[:i]) or "main"
                    cur = mats.setdefault(key, [])
                continue
            if cur is None:
                cur = mats.setdefault("rows", [])
            cur.append(s)
    return mats


@pytest.fixture
def golden():
    return read_golden
