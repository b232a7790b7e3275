import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running")


_SCENES = {}


def scene(cfg_id, **kw):
    """Cached synthetic scene (inputs only)."""
    from paper_2407_10707_amd import synth
    key = (cfg_id, tuple(sorted(kw.items())))
    if key not in _SCENES:
        _SCENES[key] = synth.make_scene(cfg_id, **kw)
    return _SCENES[key]


@pytest.fixture(scope="session")
def scene1():
    return scene(1)
