import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run")


if os.environ.get("PYTEST_XDIST_WORKER"):
    # several worker processes share the host: one intra-op thread each
    import torch
    torch.set_num_threads(1)
