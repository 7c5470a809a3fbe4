import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist, share the cores among the workers: the oracle's OpenMP loops would
# otherwise start one thread per core in every worker, and spinning threads oversubscribed
# that way slow the run down by orders of magnitude.  Set before any test loads the oracle.
if os.environ.get("PYTEST_XDIST_WORKER") and "OMP_NUM_THREADS" not in os.environ:
    _workers = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1"))
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // _workers))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long CPU-only oracle run")
