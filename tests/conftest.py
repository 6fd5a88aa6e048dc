import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    # The oracle's C half is compiled by __graft_entry__.build(); build it here
    # only when nothing is built yet.
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liblanczos_oracle.so")):
        oracle.build(force=False)
    yield
