import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as o
    o.build_library()
    yield


@pytest.fixture(scope="session", autouse=True)
def _private_tune_cache(tmp_path_factory):
    """Autotuning results of the test session go to a file of its own."""
    old = os.environ.get("TREVR_TUNE_CACHE")
    os.environ["TREVR_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "autotune.json")
    yield
    if old is None:
        os.environ.pop("TREVR_TUNE_CACHE", None)
    else:
        os.environ["TREVR_TUNE_CACHE"] = old
