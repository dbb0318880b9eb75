import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Load what is built; build only if nothing is.
_LIB = os.path.join(ROOT, "paper_1812_08606_amd", "libgmg.so")
if not os.path.exists(_LIB):
    import importlib.util

    # by path: importing the package would try to load the missing library
    _spec = importlib.util.spec_from_file_location("gmg_build", os.path.join(ROOT, "paper_1812_08606_amd", "build.py"))
    _build = importlib.util.module_from_spec(_spec)
    _spec.loader.exec_module(_build)
    _build.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    if not any("gpu" in item.keywords for item in items):
        return
    import torch

    if torch.cuda.is_available():
        return
    skip = pytest.mark.skip(reason="no HIP device in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
