"""Host side of the caller-workspace boundary (no GPU): dgp_workspace_bytes is a pure host
computation of the device bytes a plan of given sizes holds."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
torch = pytest.importorskip("torch")
from paper_0906_4548_amd import dgp  # noqa: E402


def test_workspace_bytes_sizes():
    n3, hs = 256 ** 3, 129 * 256 * 256
    f64 = dgp.workspace_bytes(256, 1, dgp.FP64)
    f32 = dgp.workspace_bytes(256, 1, dgp.FP32)
    # at least the float64 solve's fields: 3 iterates and S (real), 9 spectra
    assert f64 >= (4 * n3 * 8 + 9 * hs * 16)
    # the precision form holds the float32 solve's fields on top of the float64 ones, and its
    # force mesh in float32 instead of float64
    assert f32 >= f64 + 4 * n3 * 4 + 9 * hs * 8 - 3 * n3 * 4
    assert f64 % 256 == 0 and f32 % 256 == 0
    # the adjoint adds nine float64 fields per element
    assert dgp.workspace_bytes(256, 1, dgp.FP64, True) >= f64 + 9 * n3 * 8
    assert dgp.workspace_bytes(128, 8, dgp.FP64) > dgp.workspace_bytes(128, 1, dgp.FP64)


@pytest.mark.parametrize("n, batch, prec", [(7, 1, 0), (1024, 1, 0), (64, 0, 0), (64, 5000, 0), (64, 1, 2)])
def test_workspace_bytes_invalid_sizes(n, batch, prec):
    assert dgp.workspace_bytes(n, batch, prec) == 0
