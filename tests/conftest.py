import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def read_golden(name):
    """Rows of integers/floats from a golden fixture; '#' starts a comment."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(t) if ("." in t or "e" in t) else int(t) for t in line.split()])
    return rows


def gpu_binding():
    """The HIP binding, or skip when this machine has no GPU.  A missing
    library is an error, never a skip."""
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this machine")
    from paper_1302_4018_amd import binding
    return binding


def to_dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


import numpy as np  # noqa: E402  (used by to_dev)
