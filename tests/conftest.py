import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(scope="module")
def solver():
    """One library context on cuda:0 for a test module (GPU tests only)."""
    import torch  # noqa: F401
    from paper_2606_05687_amd import binding
    s = binding.Solver(0)
    yield s
    s.close()
