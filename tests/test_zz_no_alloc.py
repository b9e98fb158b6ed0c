"""The allocation-free deposit (dgp_deposit_noalloc) against dgp_deposit, through the C-ABI.

Two calls in a row, the second with a smaller input (a smaller mesh and fewer particles, in a
different order), each compared bit for bit with the plan-based entry point on the same input.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_0906_4548_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def _noalloc(dgp, n, box, pos):
    npart = pos.shape[1]
    grid = torch.full((n ** 3,), -7, dtype=torch.int64, device="cuda")      # stale contents on purpose
    delta = torch.full((n ** 3,), 3.5, dtype=torch.float64, device="cuda")
    st = dgp._lib.load().dgp_deposit_noalloc(int(n), float(box), ctypes.c_void_p(pos.data_ptr()),
                                             1 if pos.dtype == torch.float32 else 0, npart,
                                             ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(delta.data_ptr()),
                                             dgp._stream())
    assert st == 0, dgp._lib.load().dgp_last_error()
    return grid, delta


def _with_plan(dgp, n, box, pos):
    grid = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
    delta = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    with dgp.Plan(n, box) as plan:
        plan.deposit(pos, grid, delta)
        torch.cuda.synchronize()
    return grid, delta


def test_noalloc_deposit_matches_plan_deposit(dgp):
    cases = []
    pos, _ = inputs.zeldovich_load(64, 128.0, 3)                     # 64^3 particles on a 64^3 mesh
    cases.append((64, 128.0, torch.from_numpy(pos).cuda()))
    rng = np.random.default_rng(5)
    small = rng.uniform(0.0, 32.0, size=(3, 1001)).astype(np.float32)  # then a 16^3 mesh, 1001 particles
    cases.append((16, 32.0, torch.from_numpy(small).cuda()))
    for n, box, tp in cases:
        g0, d0 = _noalloc(dgp, n, box, tp)
        torch.cuda.synchronize()
        g1, d1 = _with_plan(dgp, n, box, tp)
        assert torch.equal(g0, g1)
        assert torch.equal(d0, d1)
        assert abs(float(d0.mean())) < 1e-14


def test_noalloc_rejects_sizes_beyond_its_limit(dgp):
    tp = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    g = torch.zeros(8, dtype=torch.int64, device="cuda")
    for n in (1024, 12):
        st = dgp._lib.load().dgp_deposit_noalloc(n, 10.0, ctypes.c_void_p(tp.data_ptr()), 0, 4,
                                                 ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(g.data_ptr()), None)
        assert st == dgp._lib.DGP_E_INVALID
