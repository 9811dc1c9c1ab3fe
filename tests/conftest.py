import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests run only where a GPU is present; on CPU hosts they are skipped
    # (select them with -m gpu on a machine with an MI355X).
    have_gpu = None
    for it in items:
        if "gpu" in it.keywords:
            if have_gpu is None:
                try:
                    import torch
                    have_gpu = bool(torch.cuda.is_available())
                except Exception:
                    have_gpu = False
            if not have_gpu:
                it.add_marker(pytest.mark.skip(reason="no GPU on this host"))
