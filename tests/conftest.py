import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_CAPTURE = None


def pytest_configure(config):
    global _CAPTURE
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")
    _CAPTURE = config.pluginmanager.getplugin("capturemanager")


def progress(msg):
    """Print a line past pytest's output capture: long GPU tests (minutes of oracle work on the
    host) report that they are alive as they go, also in a quiet run."""
    if _CAPTURE is not None:
        with _CAPTURE.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def sfac_lib():
    """The built library; built in-tree first if it is missing."""
    from paper_2209_08437_amd import sfac, build_lib
    if not os.path.exists(sfac.LIB_PATH):
        build_lib.build()
    return sfac.lib()
