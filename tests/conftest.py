"""Test configuration: the `gpu` marker and import paths.

Tests marked ``gpu`` need an MI355X and the built HIP library; everything else
runs on the CPU (the oracle, host-side logic, library loading and symbols).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    oracle.lib()
    return oracle
