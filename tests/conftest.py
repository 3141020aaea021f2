import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long statistical run")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    return oracle


@pytest.fixture(scope="session")
def flb():
    """The GPU library's Python binding (built in place if it is missing)."""
    import paper_1010_1233_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1010_1233_amd import build
        build.build()
    pkg.lib()
    return pkg
