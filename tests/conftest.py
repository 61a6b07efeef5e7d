import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU oracle cases")
    # progress notes of long GPU cases bypass output capture (see gpu_util.note)
    import gpu_util
    gpu_util.CAPTURE = config.pluginmanager.getplugin("capturemanager")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(12345)
