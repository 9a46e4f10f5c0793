import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_golden(name):
    """Parse a tests/golden text fixture: '#' comments, a bare word starts a block of number rows."""
    blocks, cur = {}, None
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            try:
                row = [float(t) for t in tok]
            except ValueError:
                cur = tok[0]
                blocks[cur] = []
                continue
            blocks[cur].append(row)
    return blocks


@pytest.fixture
def golden():
    return load_golden
