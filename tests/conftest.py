import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # load what is built; build only if nothing is
    from paper_2511_00292_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2511_00292_amd import build
        build.build()
    from oracle import build as oracle_build
    if not os.path.exists(oracle_build.LIB):
        oracle_build.build()
    from c_abi import build as c_build
    if not os.path.exists(c_build.EXE):
        c_build.build()


@pytest.fixture(scope="session")
def plain_oracle():
    from oracle import plain
    return plain._load()
