import os
import sys

# The oracle makes many small LAPACK calls; a multi-threaded BLAS spends far
# longer synchronising its threads on those than computing (a 476 x 256 QR:
# 8 ms on one thread, seconds on eight busy ones), so the tests use one.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

import pytest  # noqa: E402

try:
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # also when numpy was imported before this file
except ImportError:               # pragma: no cover
    pass

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_fraction_matrix(path):
    from fractions import Fraction
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(Fraction(t)) for t in line.split()])
    return rows
