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


def pytest_terminal_summary(terminalreporter):
    """After GPU parity runs: the largest observed FP64 log q discrepancies
    (absolute and relative) and the reduced form's per-site draw margins."""
    gh = sys.modules.get("gpu_helpers")
    if gh is None:
        return
    rows = getattr(gh, "OBSERVED_LOGQ", [])
    if rows:
        a = max(rows, key=lambda r: r[2])
        r = max(rows, key=lambda r: r[3])
        terminalreporter.write_line(f"[parity] fp64 log q over {len(rows)} comparisons: max |d| = {a[2]:.3e} "
                                    f"({a[0]}, case {a[1]}); max |d|/max(1,|log q|) = {r[3]:.3e} ({r[0]}, case {r[1]})")
    rows = getattr(gh, "OBSERVED_MARGINS", [])
    if rows:
        bad = sum(r[3] for r in rows)
        worst = max(r[4] for r in rows)
        closest = min(r[5] for r in rows)
        terminalreporter.write_line(f"[parity] reduced-form draws over {len(rows)} layers: {bad} sites differ from the "
                                    f"FP64 oracle's pick (largest margin among them {worst:.3e}); smallest margin "
                                    f"of any site {closest:.3e}")
