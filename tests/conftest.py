import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


_PROBLEMS = {}


def problem(name):
    """Session-cached synthetic problems (deterministic, seeded)."""
    import synth
    if name not in _PROBLEMS:
        makers = {
            "ico3": lambda: synth.small_icosphere(3),
            "ico4": lambda: synth.small_icosphere(4),
            "ico5": lambda: synth.config_icosphere(5),
            "torus48": lambda: synth.small_torus(48, 40),
            "torus96": lambda: synth.small_torus(96, 80),
            "torus256": lambda: synth.config_torus(256, 256),
            "pc100k": lambda: synth.small_pointcloud(100000),
            "flat": lambda: synth.small_flat_grid(40, 36),
            "pc4k": lambda: synth.small_pointcloud(4000),
            "pc20k": lambda: synth.small_pointcloud(20000),
            "hubs": lambda: synth.small_hubs(),
            "hubs_big": lambda: synth.small_hubs(256, 200),
            "torus1024": lambda: synth.config_torus(),
            "bumpy2m": lambda: synth.config_bumpy_sphere(),
        }
        _PROBLEMS[name] = makers[name]()
    return _PROBLEMS[name]


@pytest.fixture(scope="session")
def get_problem():
    return problem
