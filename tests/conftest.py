import os
import sys

import pytest

# Small Krylov problems in the oracle are dominated by BLAS thread hand-offs;
# one BLAS thread per process keeps them fast (set before numpy loads).
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: test that takes more than a few seconds")
