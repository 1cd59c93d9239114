import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer test (large inputs)")


@pytest.fixture(scope="session")
def cfg1():
    from paper_2105_13611_amd import workload
    return workload.config(1)


@pytest.fixture(scope="session")
def progress(request):
    """print(msg) past pytest's output capture, so that a long test reports
    its steps while it runs (a run that stays silent for minutes cannot be
    told from a hung one)."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is None:
            print(msg, flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(msg, flush=True)
    return say
