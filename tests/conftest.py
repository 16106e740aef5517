import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # Under pytest-xdist every worker would start one BLAS thread per core; the
    # oversubscribed spin-waiting threads slow the oracle's small dense products
    # by two orders of magnitude.  One BLAS thread per worker.
    if os.environ.get("PYTEST_XDIST_WORKER"):
        try:
            import numpy  # noqa: F401  (load the BLAS libraries first: only loaded ones are limited)
            import scipy.linalg  # noqa: F401
            import threadpoolctl
            threadpoolctl.threadpool_limits(1)
        except ImportError:
            pass
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
