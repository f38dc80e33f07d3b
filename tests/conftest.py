import os
import sys

# The oracle's many small dense factorisations run fastest on one BLAS thread.
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import pytest  # noqa: E402

try:   # also when a BLAS library was loaded before the variables above were set
    import threadpoolctl  # noqa: E402

    _BLAS_LIMIT = threadpoolctl.threadpool_limits(limits=1, user_api="blas")
except ImportError:
    _BLAS_LIMIT = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")
