import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # batched-CG autotune choices go to a cache file of this session only
    import tempfile
    os.environ.setdefault("GKO_AUTOTUNE_CACHE",
                          os.path.join(tempfile.mkdtemp(prefix="gko_tests_"), "autotune"))
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gen_mod():
    import gen
    gen.build()
    return gen


@pytest.fixture(autouse=True)
def _announce(request):
    """Name each test on the real stderr before it runs, so a GPU fault that
    kills the process still leaves the failing case in the log."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write("\n[gpu test] %s\n" % request.node.nodeid)
        sys.__stderr__.flush()
    yield
