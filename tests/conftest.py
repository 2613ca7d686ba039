import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: full-size workload, takes tens of seconds")


def _num(v):
    if v.startswith("0x"):
        return int(v, 16)
    try:
        return int(v)
    except ValueError:
        return float(v)


def load_golden(name):
    """Parse a tests/golden/*.txt fixture: 'key v1 v2 ...' lines; repeated
    keys accumulate into a list of rows."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            parsed = [_num(v) for v in vals]
            if key in out:
                if not isinstance(out[key][0], list):
                    out[key] = [out[key]]
                out[key].append(parsed)
            else:
                out[key] = parsed
    return out


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
