import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


def _lib_path():
    return os.path.join(ROOT, "paper_1511_07482_amd", "libkdefft.so")


@pytest.fixture(scope="session")
def built_lib():
    """Path of libkdefft.so, built once if absent (tests never rebuild an existing one)."""
    if not os.path.exists(_lib_path()):
        from paper_1511_07482_amd import build as _b
        _b.build()
    return _lib_path()


@pytest.fixture(scope="session")
def kf(built_lib):
    import paper_1511_07482_amd as kf_mod
    kf_mod._lib.load()
    return kf_mod


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")
