import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_sessionstart(session):
    """Build libnasg.so (hipcc cross-compiles for gfx950) when no library is
    present or when the one present was built from other sources than the
    ones in the tree (its stamp holds the hash of csrc/ and include/)."""
    from paper_2606_09794_amd import build
    if not build.is_current():
        build.build()


@pytest.fixture(scope="session")
def repo_root():
    return ROOT
