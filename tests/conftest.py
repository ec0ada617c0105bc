import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# numpy's BLAS threads busy-wait after each call and then compete with the
# oracle's OpenMP threads: the oracle's Krylov loops (many short operator calls
# between small numpy reductions) ran ten times slower.  One BLAS thread.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
import numpy  # noqa: E402,F401  (load the BLAS, then pin it)

try:
    from threadpoolctl import threadpool_limits

    threadpool_limits(1, user_api="blas")
except ImportError:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
