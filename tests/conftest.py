import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")
    # build the host-side C libraries only when nothing is built yet
    import graphgen
    import oracle
    # the mutation test runs the oracle's pins against altered copies of the
    # oracle, each built into a library of its own
    other = os.environ.get("ORACLE_LIB_UNDER_TEST")
    if other:
        oracle._LIB = other
        oracle._lib = None
    if not os.path.exists(graphgen._LIB):
        graphgen.build(force=False)
    if not os.path.exists(oracle._LIB):
        oracle.build(force=False)


def hip_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
