import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_available():
    import torch
    return torch.cuda.is_available()


# A test may load another build of the library (the host-sanitized debug
# build) in a process of its own by naming it here.
if os.environ.get("PTAFS_TEST_LIB"):
    from paper_2607_06834_amd import _lib as _ptafs_lib
    _ptafs_lib.LIB_PATH = os.environ["PTAFS_TEST_LIB"]
