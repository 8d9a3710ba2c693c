import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding (GPU tests only)."""
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2004_05197_amd import binding
    return binding


@pytest.fixture(autouse=True)
def _bounds_violations(request):
    """With CELLFFT_CHECK_BOUNDS=1 and CELLFFT_LIBRARY set to the bounds-
    checked build (build.py build_checked), every GPU test must leave the
    library's out-of-range access counter at zero: the whole GPU suite then
    doubles as a bounds check of every kernel path it reaches."""
    yield
    if os.environ.get("CELLFFT_CHECK_BOUNDS") != "1" or request.node.get_closest_marker("gpu") is None:
        return
    if not gpu_available():
        return
    from paper_2004_05197_amd import binding
    v = binding.bounds_violations()
    assert v >= 0, "CELLFFT_CHECK_BOUNDS=1 needs CELLFFT_LIBRARY set to the bounds-checked build"
    assert v == 0, f"{v} out-of-range kernel accesses counted by the bounds-checked build"
