import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# LQCD_LIBRARY=/path/liblqcd.so runs the suite against an ablation build
# (python -m paper_2001_07557_amd.build -D ... --out DIR); default: in-tree.
if os.environ.get("LQCD_LIBRARY"):
    from paper_2001_07557_amd import _lib as _lqcd_lib
    _lqcd_lib.LIB_PATH = os.path.abspath(os.environ["LQCD_LIBRARY"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session")
def root():
    return ROOT
