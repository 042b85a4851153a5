import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "oracle_job(name): the test waits for a background oracle job")


def pytest_collection_finish(session):
    """Start the background oracle jobs of the selected tests (only where a
    GPU is present: the tests that wait for them need one)."""
    names = []
    for item in session.items:
        m = item.get_closest_marker("oracle_job")
        if m:
            names.extend(a for a in m.args if a not in names)
    if not names:
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
    except ImportError:
        return
    import oracle_jobs
    for name in names:
        oracle_jobs.start(name)
