import os
import sys

import pytest

# torch first: its HIP runtime must be the one in the process before the
# library (which links the system HIP runtime) is loaded, or torch's own
# device initialisation can fail later in the same process
try:
    import torch  # noqa: F401
except ImportError:  # the CPU suite runs without it
    torch = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the batch autotuner keeps its choices in a file: tests use one of their own
if "CG_TUNE_CACHE" not in os.environ:
    import tempfile

    os.environ["CG_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="cg_tune_"), "tune.txt")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_c():
    from oracle import native

    native.build(force=False)
    return native
