import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on the device)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build(force=False)
    yield


@pytest.fixture(scope="session")
def hip_lib_built():
    """The HIP library is built in-tree by __graft_entry__.build(); build it here if it is missing."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("gmp_build", os.path.join(ROOT, "paper_1606_00519_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB
