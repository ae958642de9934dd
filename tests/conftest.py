import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The mutant tests point this at a folder holding a deliberately broken copy of the
# Python oracle package, to check that the pins catch the planted mistake.
_PY_ORACLE_ROOT = os.environ.get("VESNET_ORACLE_PY_ROOT")
if _PY_ORACLE_ROOT:
    sys.path.insert(0, _PY_ORACLE_ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; run through the C-ABI library")


def pytest_runtest_setup(item):
    if "gpu" in item.keywords:
        import torch
        if not torch.cuda.is_available():
            pytest.skip("no GPU visible")
