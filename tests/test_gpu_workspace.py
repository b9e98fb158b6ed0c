"""Plans on a caller-owned device workspace (dgp_plan_create_ws) against plans that allocate their
own: the same kernels on the same inputs, so the outputs are identical to the bit; the byte
query equals what a plan holds; too small, misaligned and adjoint-less workspaces are refused."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cosmology as cos, pm  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import OM0, to_dev, calibrate_lambda, gpu_params  # noqa: E402


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ws(dgp, n, batch, prec, adjoint):
    return torch.empty(dgp.workspace_bytes(n, batch, prec, adjoint), dtype=torch.uint8, device="cuda")


def test_device_bytes_equal_the_query(dgp):
    say("workspace: device bytes")
    for prec in (dgp.FP64, dgp.FP32):
        with dgp.Plan(64, 128.0, precision=prec) as plan:
            assert plan.device_bytes() == dgp.workspace_bytes(64, 1, prec)
    n, box, B = 16, 32.0, 2
    d = torch.from_numpy(np.stack([inputs.lognormal_delta(n, box, 0.5, 60 + b) for b in range(B)])).to("cuda")
    with dgp.Plan(n, box, batch=B) as plan:
        u = torch.zeros_like(d)
        st, _ = plan.solve_field(gpu_params(dgp, lam=0.5, tol=1e-12, max_iter=100), d, u)
        assert st == 0
        gd = torch.zeros_like(d)
        plan.solve_field_backward(gpu_params(dgp, lam=0.5, tol=1e-12, max_iter=100), d, u, torch.ones_like(d), gd)
        assert plan.device_bytes() == dgp.workspace_bytes(n, B, dgp.FP64, True)


@pytest.mark.parametrize("prec", [0, 1])
def test_workspace_plan_solve_and_backward_identical(dgp, prec):
    say("workspace: solve and backward", prec)
    n, box = 32, 64.0
    delta = inputs.lognormal_delta(n, box, 1.0, 61)
    lam = calibrate_lambda(delta, box, 3.0)
    prm = gpu_params(dgp, lam=lam, tol=1e-10, max_iter=100)
    d = to_dev(delta)
    g = torch.from_numpy(np.random.default_rng(62).standard_normal(n ** 3)).to("cuda")
    outs = []
    for ws in (None, _ws(dgp, n, 1, prec, True)):
        with dgp.Plan(n, box, precision=prec, workspace=ws) as plan:
            u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            st, info = plan.solve_field(prm, d, u)
            assert st == 0
            gd = torch.zeros_like(u)
            st2, _ = plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12, max_iter=100), d, u, g, gd)
            assert st2 == 0
            if ws is not None:
                assert plan.device_bytes() <= ws.numel()
            torch.cuda.synchronize()
            outs.append((u.cpu().numpy(), gd.cpu().numpy(), info[0]["iters"]))
    assert outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_workspace_plan_step_identical(dgp):
    say("workspace: PM step")
    n, box, a, dlna = 32, 64.0, 0.5, 0.005
    pos, psi = inputs.zeldovich_load(n, box, 63, dtype=np.float32)
    c = cos.coefficients(OM0, a)
    vel = (a * a * c.E * cos.omega_m_of_a(OM0, a) ** 0.55 * psi).astype(np.float32)
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 1.78)
    outs = []
    for ws in (None, _ws(dgp, n, 1, dgp.FP32, False)):
        with dgp.Plan(n, box, precision=dgp.FP32, workspace=ws) as plan:
            tp, tv = to_dev(pos, torch.float32), to_dev(vel, torch.float32)
            u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            st, _ = plan.step(gpu_params(dgp, lam=lam, tol=1e-10), tp, tv, u, dlna)
            assert st == 0
            torch.cuda.synchronize()
            outs.append((tp.cpu().numpy(), tv.cpu().numpy(), u.cpu().numpy()))
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_workspace_refusals(dgp):
    say("workspace: refusals")
    n, box = 16, 32.0
    need = dgp.workspace_bytes(n, 1, dgp.FP64)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(dgp._lib.DGPError):
        dgp.Plan(n, box, workspace=small)
    big = torch.empty(need + 1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(dgp._lib.DGPError):
        dgp.Plan(n, box, workspace=big[128:])   # not 256-byte aligned
    # sized without the adjoint: the solve runs, the backward is refused before any work
    ws = _ws(dgp, n, 1, dgp.FP64, False)
    delta = to_dev(inputs.lognormal_delta(n, box, 0.5, 64))
    with dgp.Plan(n, box, workspace=ws) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, _ = plan.solve_field(gpu_params(dgp, lam=0.5, tol=1e-12, max_iter=100), delta, u)
        assert st == 0
        gd = torch.zeros_like(u)
        with pytest.raises(dgp._lib.DGPError):
            plan.solve_field_backward(gpu_params(dgp, lam=0.5, tol=1e-12, max_iter=100), delta, u, torch.ones_like(u), gd)
        st, _ = plan.solve_field(gpu_params(dgp, lam=0.5, tol=1e-12, max_iter=100), delta, u)   # still usable
        assert st == 0
