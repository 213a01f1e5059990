import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running host test")


@pytest.fixture(autouse=True)
def _tuning_follows_environment(request):
    # A GPU test may change DSLASH_* tuning variables (monkeypatch restores
    # them at its end); the library reads them once per process, so it reads
    # them again after the test.  Autouse: set up before, torn down after, the
    # test's monkeypatch.
    yield
    mod = sys.modules.get("paper_1808_05506_amd.dslash")
    if request.node.get_closest_marker("gpu") is not None and mod is not None:
        mod.reload_tuning()
