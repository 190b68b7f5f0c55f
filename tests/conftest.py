import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU statistics test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O

    if not os.path.exists(O.LIB):
        O.build()
    return O


@pytest.fixture(scope="session")
def W():
    from paper_2502_06319_amd import workloads

    return workloads


ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="session")
def eng():
    """One HIP context on device 0 for the GPU tests (fails loudly without one)."""
    from paper_2502_06319_amd import cosmica

    e = cosmica.Engine(0)
    yield e
    e.close()


@pytest.fixture(scope="session")
def othreads():
    return ORACLE_THREADS
