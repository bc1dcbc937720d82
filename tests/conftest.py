import os
import sys

import numpy  # noqa: F401  (loads the BLAS library that the limit below applies to)
import pytest
from threadpoolctl import threadpool_limits

# The checker's C code parallelises with OpenMP; numpy's BLAS threads, which
# spin after every small product of the Krylov loops, would compete with it for
# the same cores (a 40x slowdown of the checker's Lanczos at N = 20).
threadpool_limits(1, user_api="blas")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side checks")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import native
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        native.build(force=True)
    return native
