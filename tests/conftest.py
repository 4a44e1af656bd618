"""Shared test configuration: the `gpu` marker and common fixtures."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: runs on an MI355X through the C-ABI library")
    config.addinivalue_line("markers", "slow: statistical test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle, built once per session."""
    import oracle
    from oracle import build
    build.build(force=False)
    return oracle
