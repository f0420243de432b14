import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side test (oracle on larger inputs)")


def golden_path(name):
    return os.path.join(ROOT, "tests", "golden", name)


def read_golden(name):
    """Parse a tests/golden text fixture: 'key v1 v2 ...' lines, 'row r: c=v ...' lines and
    'dense ...' lines; '#' starts a comment."""
    out = {"rows": {}, "dense": []}
    with open(golden_path(name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("row "):
                head, rest = line.split(":", 1)
                r = int(head.split()[1])
                out["rows"][r] = [(int(a), float(b)) for a, b in (t.split("=") for t in rest.split())]
            elif line.startswith("dense "):
                out["dense"].append([float(t) for t in line.split()[1:]])
            else:
                k, *vals = line.split()
                out[k] = [float(v) if "." in v else int(v) for v in vals]
    return out
