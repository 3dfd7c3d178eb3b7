import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly when it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a visible GPU")
    import paper_2110_01481_amd as abg
    abg.load_library()
    return abg


def pytest_sessionfinish(session, exitstatus):
    """Releases the library's engines, geometries and process-wide resources while the
    HIP runtime is still up (only if a test loaded the library)."""
    mod = sys.modules.get("paper_2110_01481_amd._binding")
    if mod is not None and mod._lib is not None:
        mod.shutdown()
