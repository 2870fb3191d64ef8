import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def fig2():
    """The worked example of the paper (Fig. 2): edges (0-based), raw, net."""
    path = os.path.join(ROOT, "tests", "golden", "fig2_example.txt")
    sec, data = None, {"edges": [], "raw": [], "net": []}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                sec = line.strip("[]")
                continue
            vals = [int(x) for x in line.split()]
            if sec == "edges":
                data["edges"].append((vals[0] - 1, vals[1] - 1))
            else:
                data[sec].append(vals[1:])
    import numpy as np
    return {
        "n": 6,
        "edges": data["edges"],
        "raw": np.array(data["raw"], dtype=np.int64),
        "net": np.array(data["net"], dtype=np.int64),
    }


@pytest.fixture(scope="session")
def table2():
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "table2_u16.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return np.array(rows, dtype=np.int64)
