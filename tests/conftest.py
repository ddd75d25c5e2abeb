import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for _p in (ROOT, os.path.join(ROOT, "tests", "golden")):
    if _p not in sys.path:
        sys.path.insert(0, _p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: statistical checks that take tens of seconds")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle
    oracle.build()
    return oracle


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    # Name the case before any GPU work so that a run that loses the box
    # still says which test it was in.
    if request.node.get_closest_marker("gpu") is not None:
        print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


@pytest.fixture(scope="session")
def rfim_mod():
    import paper_1508_06268_amd as P
    P.load_library()
    return P
