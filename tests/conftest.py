import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Every knob the library reads, created (empty: the library's default) before any test touches
# the device, so that tests later only replace values (gpu_util.env) and never add or remove a
# name while the device runtime's threads may call getenv.
KNOBS = ("ESWAVE_CG_FUSED", "ESWAVE_FORCE_VARIANT", "ESWAVE_FUSE_UP2", "ESWAVE_NO_REVERSE", "ESWAVE_PERSIST_SPIN",
         "ESWAVE_PLAN_BRANCHES", "ESWAVE_PLAN_CHUNK", "ESWAVE_PLAN_COARSE_MAX", "ESWAVE_PLAN_LAG",
         "ESWAVE_PLAN_PERSISTENT", "ESWAVE_SPLIT_MIN", "ESWAVE_STREAMED", "ESWAVE_STREAMS", "ESWAVE_TAIL_MAX",
         "ESWAVE_TUNE_CACHE")
for _k in KNOBS:
    os.environ.setdefault(_k, "")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def lib():
    """The built C-ABI library loaded through the Python binding (no device call)."""
    from paper_2507_02401_amd import _lib
    return _lib.load()
