import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libsagms")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_pool():
    """A pool of host processes for oracle runs (spawned, so they never touch
    the GPU): SAGMS_ORACLE_PROCS workers, default the host's cores up to 16."""
    import multiprocessing as mp
    helpers = os.path.join(os.path.dirname(os.path.abspath(__file__)), "helpers")
    if helpers not in sys.path:
        sys.path.insert(0, helpers)
    procs = int(os.environ.get("SAGMS_ORACLE_PROCS", min(16, os.cpu_count() or 1)))
    with mp.get_context("spawn").Pool(procs) as pool:
        yield pool
