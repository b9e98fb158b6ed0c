"""GPU adjoints (implicit solve adjoint, CIC adjoint, P(k) adjoint) against the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import field as fld, pm, power, adjoint  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import OM0, to_dev, oracle_params, calibrate_lambda, gpu_params, rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_solve_adjoint_matches_oracle(dgp, n):
    say("adjoint", n)
    box = 2.0 * n
    delta = inputs.lognormal_delta(n, box, 1.0, 40 + n)
    lam = calibrate_lambda(delta, box, 3.0)
    op = oracle_params(lam=lam, tol=1e-13, max_iter=200)
    u, _ = fld.solve(delta, box, op)
    g = np.random.default_rng(n).standard_normal((n, n, n))
    mu_ref, gd_ref, hist = adjoint.adjoint_picard(u, g, box, op, tol=1e-12)
    with dgp.Plan(n, box) as plan:
        gd = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12, max_iter=200), to_dev(delta),
                                             to_dev(u), to_dev(g), gd)
        assert st == 0 and info[0]["iters"] == len(hist) - 1
        assert rel_l2(gd.cpu().numpy().reshape(n, n, n), gd_ref) <= 1e-10
    if n == 8:
        _, gd_dense = adjoint.adjoint_dense(u, g, box, op)
        assert rel_l2(gd.cpu().numpy().reshape(n, n, n), gd_dense) <= 1e-10


def test_deposit_and_power_adjoints(dgp):
    say("cic / power adjoints")
    n, box = 16, 32.0
    pos, _ = inputs.zeldovich_load(n, box, 9)
    rng = np.random.default_rng(3)
    gmesh = rng.standard_normal((n, n, n))
    ref = adjoint.deposit_backward(pos, gmesh, box)
    field = inputs.gaussian_field(n, box, 4)
    gpk = rng.standard_normal(64)
    ref_p = power.power_spectrum_grad(fld.c_from_u(field, box, oracle_params()), gpk, box)
    ref_p = fld.c_from_u(ref_p, box, oracle_params())
    with dgp.Plan(n, box) as plan:
        gp = torch.zeros((3, pos.shape[1]), dtype=torch.float64, device="cuda")
        plan.deposit_backward(to_dev(pos), to_dev(gmesh), gp)
        assert rel_l2(gp.cpu().numpy(), ref) <= 1e-13
        gf = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.power_spectrum_backward(gpu_params(dgp), to_dev(field), gpk, gf, of_c=True)
        assert rel_l2(gf.cpu().numpy().reshape(n, n, n), ref_p) <= 1e-10


def test_autograd_chain_against_oracle_and_fd(dgp):
    """positions -> deposit -> solve -> P_C(k) -> loss; gradient against the oracle chain and central FD."""
    say("autograd chain")
    from paper_0906_4548_amd.autograd import CICDeposit, FieldSolve, PowerOfC, power_loss
    n, box = 16, 32.0
    pos, _ = inputs.zeldovich_load(n, box, 11, rms_disp=1.5)
    _, delta0 = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta0, box, 1.0)
    op = oracle_params(lam=lam, tol=1e-13, max_iter=200)
    u0, _ = fld.solve(delta0, box, op)
    pk0, _, _ = power.power_spectrum(fld.c_from_u(u0, box, op), box)
    target = pk0 * 1.1
    wts = np.where(pk0 > 0, 1.0 / np.where(pk0 > 0, pk0, 1.0) ** 2, 0.0)
    # oracle gradient wrt positions
    loss_ref, gu = adjoint.c_power_loss(u0, box, op, target, wts)
    _, gd, _ = adjoint.adjoint_picard(u0, gu, box, op, tol=1e-13)
    gpos_ref = adjoint.deposit_backward(pos, gd, box)
    with dgp.Plan(n, box) as plan:
        prm = gpu_params(dgp, lam=lam, tol=1e-13, max_iter=200)
        tp = to_dev(pos).requires_grad_(True)
        delta = CICDeposit.apply(tp, plan)
        u = FieldSolve.apply(delta, plan, prm)
        pk = PowerOfC.apply(u, plan, prm)
        loss = power_loss(pk[0], to_dev(target), to_dev(wts))
        loss.backward()
        assert abs(loss.item() - loss_ref) <= 1e-9 * abs(loss_ref)
        gpos = tp.grad.cpu().numpy()
        assert rel_l2(gpos, gpos_ref) <= 1e-9
        # central differences on a few particles (away from grid planes), step 1e-4 Mpc/h
        h = 1e-4
        idx = np.random.default_rng(12).choice(pos.shape[1], 4, replace=False)
        for p in idx:
            for d in range(3):
                s = pos[d, p] * n / box
                if abs(s - np.round(s)) < 2e-3:
                    continue
                vals = []
                for sgn in (1, -1):
                    q = pos.copy()
                    q[d, p] += sgn * h
                    with torch.no_grad():
                        dl = CICDeposit.apply(to_dev(q), plan)
                        uu = FieldSolve.apply(dl, plan, prm)
                        vals.append(power_loss(PowerOfC.apply(uu, plan, prm)[0], to_dev(target), to_dev(wts)).item())
                fd = (vals[0] - vals[1]) / (2 * h)
                assert abs(fd - gpos[d, p]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(gpos)))
