import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    return O


def load_binding():
    """The ctypes binding; builds libising.so first when it is missing.

    On a machine with a GPU a build or load failure is an error, never a
    skip, so that no GPU test can pass without the HIP library."""
    try:
        from paper_2311_09275_amd import binding
        return binding
    except ImportError:
        from paper_2311_09275_amd import build
        build.build()
        from paper_2311_09275_amd import binding
        return binding
