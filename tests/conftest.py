import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# The oracle's products are small (at most a few hundred rows by a few dozen columns):
# BLAS threads only contend on them (one thread is 13-25x faster on 8 cores), so the
# tests run the oracle single-threaded.
try:
    from threadpoolctl import threadpool_limits

    _BLAS_LIMIT = threadpool_limits(limits=1, user_api="blas")
except Exception:  # threadpoolctl missing: the default thread count is only slower
    _BLAS_LIMIT = None
