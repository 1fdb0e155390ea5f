import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    """The C-ABI library loaded through the Python binding (GPU tests only)."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_1707_08369_amd as svdu
    return svdu


@pytest.fixture(autouse=True)
def _tile_shape_from_env(request):
    """SVDU_TEST_TILE_SHAPE=k runs the GPU tests with the product kernels forced to tile shape k."""
    v = os.environ.get("SVDU_TEST_TILE_SHAPE")
    if not v or request.node.get_closest_marker("gpu") is None:
        yield
        return
    import paper_1707_08369_amd as svdu
    old = svdu.set_option(svdu.SVDU_OPT_TILE_SHAPE, int(v))
    yield
    svdu.set_option(svdu.SVDU_OPT_TILE_SHAPE, old)
