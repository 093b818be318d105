import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU statistical test")


@pytest.fixture(autouse=True)
def _single_thread_blas():
    """Keep numpy's BLAS single-threaded so the CPU suite behaves the same everywhere."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        yield
        return
    with threadpool_limits(1):
        yield


def pytest_collection_finish(session):
    """torch bundles a HIP runtime of its own beside the one libtnmc links
    against; in one process, torch's must initialise first or it finds no GPU.
    GPU sessions therefore touch torch's runtime before any test runs."""
    if any(item.get_closest_marker("gpu") for item in session.items):
        try:
            import torch
        except ImportError:  # pragma: no cover
            return
        torch.cuda.is_available()
