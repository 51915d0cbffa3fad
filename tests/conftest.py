import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle case")


_SYSTEMS = {}


def cached_system(name, **kw):
    """Generate (once per session) one of the named synthetic systems."""
    from synth import build_system, configs
    key = (name, tuple(sorted(kw.items())))
    if key not in _SYSTEMS:
        _SYSTEMS[key] = build_system(configs.BY_NAME[name](**kw))
    return _SYSTEMS[key]


@pytest.fixture(scope="session")
def small_dense():
    return cached_system("small_dense")


@pytest.fixture(scope="session")
def small_trunc():
    return cached_system("small_trunc")


@pytest.fixture(scope="session")
def separated():
    return cached_system("separated")


@pytest.fixture(scope="session")
def small_odd():
    return cached_system("small_odd")


@pytest.fixture(scope="session")
def small_kt():
    return cached_system("small_kt")


@pytest.fixture(scope="session")
def small_kt_exactp():
    return cached_system("small_kt_exactp")
