import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# the oracle factors many small matrices; BLAS threading only adds overhead there
os.environ.setdefault("OPENBLAS_NUM_THREADS", os.environ.get("SFLS_TEST_BLAS_THREADS", "1"))
try:
    import numpy  # noqa: F401  (load both BLAS copies before limiting them)
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits

    threadpool_limits(int(os.environ.get("SFLS_TEST_BLAS_THREADS", "1")))
except Exception:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")
