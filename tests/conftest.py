import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# the mutation test runs the oracle's pins against altered copies of the
# oracle package, each in a directory of its own
ORACLE_COPY = os.environ.get("ORACLE_PKG_DIR")
if ORACLE_COPY:
    sys.path.insert(0, ORACLE_COPY)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")
    # build the host-side C libraries only when nothing is built yet
    import graphgen
    import oracle
    if ORACLE_COPY and not os.path.abspath(oracle.__file__).startswith(os.path.abspath(ORACLE_COPY) + os.sep):
        raise RuntimeError("ORACLE_PKG_DIR is set but oracle was imported from %s" % oracle.__file__)
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
