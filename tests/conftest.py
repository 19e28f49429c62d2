import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running check (large grids)")



def pytest_sessionstart(session):
    # lets tests.gpu_helpers.progress print past the output capture
    import tests.gpu_helpers as helpers
    helpers.CAPTURE_MANAGER = session.config.pluginmanager.getplugin("capturemanager")
