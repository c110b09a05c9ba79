import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs through the HIP C-ABI")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import binding
    if not os.path.exists(binding.LIB_PATH):
        binding.build(force=False)
