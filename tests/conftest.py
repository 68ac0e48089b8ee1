import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large inputs")
    # Build the libraries once if nothing is built yet (CPU-only compile).
    from paper_1503_07881_amd import build as pkg_build
    import oracle
    pkg_dir = os.path.dirname(pkg_build.__file__)
    if not all(os.path.exists(os.path.join(pkg_dir, lib)) for lib in pkg_build.LIBS):
        pkg_build.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(params=["sort", "hash", "hash_parts"])
def method(request):
    """Runs the test once per node-numbering method (every size bucket set to
    it), restoring the library's schedule afterwards.  hash_parts is the hash
    numbering through keys grouped by table part, at every table size."""
    from paper_1503_07881_amd import ringo
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    ringo.set_node_method(ringo.NODES_SORT if request.param == "sort" else ringo.NODES_HASH)
    os.environ["RINGO_HASH_PARTS"] = "1" if request.param == "hash_parts" else "0"
    yield request.param
    os.environ.pop("RINGO_HASH_PARTS", None)
    for e, (d, it, m) in enumerate(saved):
        ringo.tune_set(1 << e, d, it, m)


@pytest.fixture(params=["lds", "pipeline"])
def small_path(request):
    """Runs the test with the default routing (tables of at most 2048 rows
    converted in LDS, single tables up to 2^20 rows numbered by sorting on the
    sync-free path) and with every table sent through the pass pipeline."""
    if request.param == "pipeline":
        os.environ["RINGO_SMALL_TABLES"] = "0"
        os.environ["RINGO_FIXED_PATH"] = "0"
    yield request.param
    os.environ.pop("RINGO_SMALL_TABLES", None)
    os.environ.pop("RINGO_FIXED_PATH", None)
