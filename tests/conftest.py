import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def golden_rows(name):
    """Non-comment, non-blank lines of a golden fixture, split on whitespace."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


def say(*args):
    """Names the case about to touch the GPU, flushed before it runs."""
    print("[case]", *args, flush=True)


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding on cuda:0; fails (never falls back) without it."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2408_06213_amd import brr

    torch.cuda.set_device(0)
    return brr


def to_dev(a):
    import numpy as np
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()
