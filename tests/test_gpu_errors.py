"""Error paths and degenerate cases of the C-ABI on the GPU.

Non-finite inputs are rejected with DGP_E_INVALID; max_iter exhaustion returns DGP_NOT_CONVERGED
with the minimum-residual iterate (Sec. III C stopping rule, as in the oracle); a uniform density
has the exact solution u = 0; the implicit adjoint refuses a field with bad-point vertices and
autograd refuses to differentiate a solve that did not converge.  Every case is forced from the
host through its inputs: every kernel runs to its normal end.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import field as fld, adjoint  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import to_dev, oracle_params, calibrate_lambda, gpu_params, rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_nonfinite_delta_is_invalid(dgp, prec, bad):
    say("nonfinite delta", prec, bad)
    n, box = 16, 32.0
    delta = inputs.lognormal_delta(n, box, 1.0, 3)
    delta[3, 4, 5] = float(bad)
    with dgp.Plan(n, box, batch=2, precision=prec) as plan:
        d = to_dev(np.stack([inputs.lognormal_delta(n, box, 1.0, 4), delta]))
        u = torch.zeros_like(d)
        infos = (dgp._lib.Info * 2)()
        import ctypes
        st = dgp._lib.load().dgp_solve_field(plan.handle, ctypes.byref(gpu_params(dgp, lam=1.0, tol=1e-8)),
                                             ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(u.data_ptr()), None, infos,
                                             dgp._stream())
        assert st == dgp._lib.DGP_E_INVALID
        assert b"non-finite" in dgp._lib.load().dgp_last_error()
        assert infos[1].status == dgp._lib.DGP_E_INVALID and infos[0].status == 0
        # the plan stays usable
        st, info = plan.solve_field(gpu_params(dgp, lam=1.0, tol=1e-8), d[:1].repeat(2, 1, 1, 1).contiguous(), u)
        assert st == 0


def test_nonfinite_warm_start_is_invalid(dgp):
    say("nonfinite warm start")
    n, box = 16, 32.0
    with dgp.Plan(n, box) as plan:
        d = to_dev(inputs.lognormal_delta(n, box, 1.0, 3))
        u = torch.zeros_like(d)
        u[7, 7, 7] = float("nan")
        with pytest.raises(dgp._lib.DGPError) as e:
            plan.solve_field(gpu_params(dgp, lam=1.0, tol=1e-8, init=dgp.INIT_WARM), d, u)
        assert e.value.code == dgp._lib.DGP_E_INVALID


@pytest.mark.parametrize("fp32", [False, True])
def test_nonfinite_position(dgp, fp32):
    say("nonfinite position", fp32)
    n, box = 16, 32.0
    pos, psi = inputs.zeldovich_load(n, box, 5)
    pos = pos.astype(np.float32 if fp32 else np.float64)
    pos[1, 100] = np.nan
    dt = torch.float32 if fp32 else torch.float64
    with dgp.Plan(n, box) as plan:
        tp = to_dev(pos, dt)
        d = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.deposit(tp, None, d)
        assert bool(torch.all(torch.isnan(d)))
        with pytest.raises(dgp._lib.DGPError) as e:
            plan.solve_field(gpu_params(dgp, lam=1.0, tol=1e-8), d, torch.zeros_like(d))
        assert e.value.code == dgp._lib.DGP_E_INVALID
        for mode in (dgp.FORCE_NLDGP, dgp.FORCE_GRH):
            with pytest.raises(dgp._lib.DGPError) as e:
                plan.step(gpu_params(dgp, lam=1.0, tol=1e-8, force_mode=mode), tp, to_dev(0.1 * psi, dt),
                          torch.zeros_like(d), 0.005)
            assert e.value.code == dgp._lib.DGP_E_INVALID


@pytest.mark.parametrize("prec", [0, 1])
def test_uniform_density_gives_zero(dgp, prec):
    """A perfect lattice deposits delta = 0 exactly: S = 0, eps = 0, u = 0 with zero updates."""
    say("uniform", prec)
    n, box = 16, 32.0
    q1 = (np.arange(n) + 0.5) * box / n
    qx, qy, qz = np.meshgrid(q1, q1, q1, indexing="ij")
    lat = np.stack([qx.ravel(), qy.ravel(), qz.ravel()])
    with dgp.Plan(n, box, precision=prec) as plan:
        d = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.deposit(to_dev(lat), None, d)
        assert bool(torch.all(d == 0))
        u = torch.full_like(d, 3.0)
        st, info = plan.solve_field(gpu_params(dgp, lam=2.0, tol=1e-10), d, u)
        assert st == 0 and info[0]["iters"] == 0 and info[0]["resid"] == 0.0 and info[0]["eps"] == 0.0
        assert bool(torch.all(u == 0))


def _c1(n=32, box=64.0, seed=1, rnl=3.0):
    delta = inputs.lognormal_delta(n, box, 1.0, seed)
    return delta, calibrate_lambda(delta, box, rnl)


@pytest.mark.parametrize("prec", [0, 1])
def test_max_iter_returns_min_residual_iterate(dgp, prec):
    """tol out of reach: the solve stops at max_iter with DGP_NOT_CONVERGED and returns the
    minimum-residual iterate, the oracle's choice under the same rule."""
    say("max_iter", prec)
    n, box = 32, 64.0
    delta, lam = _c1(n, box)
    k = 4
    u_ref, iref = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-15, max_iter=k))
    assert iref.status == fld.STATUS_NOT_CONVERGED
    with dgp.Plan(n, box, precision=prec) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-15, max_iter=k), to_dev(delta), u)
        assert st == dgp._lib.DGP_NOT_CONVERGED and info[0]["status"] == st
        got = u.cpu().numpy().reshape(n, n, n)
        if prec == 0:
            assert info[0]["iters"] == iref.iters
            assert abs(info[0]["resid"] - iref.resid) <= 1e-12 * iref.resid
            assert rel_l2(got, u_ref) <= 1e-12
        else:   # float32 updates: the iterate to the float32 bar
            assert rel_l2(got, u_ref) <= 1e-5


def test_adjoint_rejects_vertex_points(dgp):
    """A field holding the vertex value -alpha/(2 (1-w) lam) of a bad point has D = 0 there."""
    say("adjoint vertex")
    n, box = 16, 32.0
    delta, lam = _c1(n, box, seed=5, rnl=1.0)
    u, _ = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-12))
    prm = oracle_params(lam=lam)
    u[2, 3, 4] = -prm.alpha / (2.0 * (1.0 - prm.w) * lam)
    g = np.random.default_rng(3).standard_normal(u.shape)
    with dgp.Plan(n, box) as plan:
        gd = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        with pytest.raises(dgp._lib.DGPError) as e:
            plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12), to_dev(delta), to_dev(u), to_dev(g), gd)
        assert e.value.code == dgp._lib.DGP_E_INVALID and b"2 (1-w) lam u + alpha <=" in dgp._lib.load().dgp_last_error()
        g[0, 0, 0] = float("nan")
        u2, _ = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-12))
        with pytest.raises(dgp._lib.DGPError):
            plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12), to_dev(delta), to_dev(u2), to_dev(g), gd)


@pytest.mark.parametrize("k", [0, 1, 3])
def test_adjoint_max_iter(dgp, k):
    """The transposed relaxation stopped at max_iter returns DGP_NOT_CONVERGED and the
    minimum-residual mu; here the residual decreases monotonically, so that is the oracle's
    mu after the same number of updates (k = 0: the first multiplier g / D itself)."""
    say("adjoint max_iter", k)
    n, box = 16, 32.0
    delta, lam = _c1(n, box, seed=6, rnl=3.0)
    op = oracle_params(lam=lam, tol=1e-13, max_iter=200)
    u, _ = fld.solve(delta, box, op)
    g = np.random.default_rng(4).standard_normal(u.shape)
    _, gd_ref, hist = adjoint.adjoint_picard(u, g, box, op, tol=0.0, max_iter=k + 1)
    assert all(a > b for a, b in zip(hist, hist[1:]))
    with dgp.Plan(n, box) as plan:
        gd = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-15, max_iter=k), to_dev(delta),
                                             to_dev(u), to_dev(g), gd)
        assert st == dgp._lib.DGP_NOT_CONVERGED and info[0]["iters"] == k
        assert abs(info[0]["resid"] - hist[k]) <= 1e-10 * hist[k]
        _, gd_k, _ = adjoint.adjoint_picard(u, g, box, op, tol=0.0, max_iter=k)
        assert rel_l2(gd.cpu().numpy().reshape(n, n, n), gd_k) <= 1e-11


def test_adjoint_batch_stops_per_element(dgp):
    """A batch whose elements stop at different iterations: the easy field converges and returns its
    converged multiplier while the other, still running, stops at max_iter with its own
    minimum-residual multiplier; each against the oracle's transposed relaxation of that field."""
    say("adjoint batch stops")
    n, box = 16, 32.0
    d_easy = inputs.lognormal_delta(n, box, 0.3, 21)
    d_hard = inputs.lognormal_delta(n, box, 3.0, 22)
    lam = calibrate_lambda(d_hard, box, 3.0)
    op = oracle_params(lam=lam, tol=1e-13, max_iter=200)
    us = [fld.solve(d, box, op)[0] for d in (d_easy, d_hard)]
    rng = np.random.default_rng(23)
    gs = [rng.standard_normal((n, n, n)) for _ in range(2)]
    with dgp.Plan(n, box, batch=2) as plan:
        args = (to_dev(np.stack([d_easy, d_hard])), to_dev(np.stack(us)), to_dev(np.stack(gs)))
        gd = torch.zeros((2, n ** 3), dtype=torch.float64, device="cuda")
        st, info = plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12, max_iter=200), *args, gd)
        assert st == 0
        i_easy, i_hard = info[0]["iters"], info[1]["iters"]
        assert i_easy + 2 <= i_hard, (i_easy, i_hard)
        m = (i_easy + i_hard) // 2
        st, info = plan.solve_field_backward(gpu_params(dgp, lam=lam, tol=1e-12, max_iter=m), *args, gd)
        assert st == dgp._lib.DGP_NOT_CONVERGED
        assert info[0]["status"] == 0 and info[0]["iters"] == i_easy
        assert info[1]["status"] == dgp._lib.DGP_NOT_CONVERGED and info[1]["iters"] == m
        got = gd.cpu().numpy().reshape(2, n, n, n)
        _, ref_easy, _ = adjoint.adjoint_picard(us[0], gs[0], box, op, tol=1e-12, max_iter=200)
        assert rel_l2(got[0], ref_easy) <= 1e-10
        _, ref_hard, _ = adjoint.adjoint_picard(us[1], gs[1], box, op, tol=0.0, max_iter=m)
        _, _, hist = adjoint.adjoint_picard(us[1], gs[1], box, op, tol=0.0, max_iter=m + 1)
        assert all(a > b for a, b in zip(hist, hist[1:]))   # the minimum-residual multiplier is the last
        # (the residual is a difference of O(1) terms: its float64 rounding floor is ~1e-16 absolute)
        assert abs(info[1]["resid"] - hist[m]) <= 1e-10 * hist[m] + 1e-14
        assert rel_l2(got[1], ref_hard) <= 1e-11


def test_autograd_refuses_unconverged_solve(dgp):
    say("autograd unconverged")
    from paper_0906_4548_amd.autograd import FieldSolve, SolveNotConvergedError
    n, box = 16, 32.0
    delta, lam = _c1(n, box, seed=7)
    with dgp.Plan(n, box) as plan:
        d = to_dev(delta).requires_grad_(True)
        with pytest.warns(RuntimeWarning):
            u = FieldSolve.apply(d, plan, gpu_params(dgp, lam=lam, tol=1e-15, max_iter=2))
        with pytest.raises(SolveNotConvergedError):
            torch.sum(u * u).backward()
        d2 = to_dev(delta).requires_grad_(True)
        u2 = FieldSolve.apply(d2, plan, gpu_params(dgp, lam=lam, tol=1e-12, max_iter=200),
                              gpu_params(dgp, lam=lam, tol=1e-15, max_iter=2))
        with pytest.raises(SolveNotConvergedError):
            torch.sum(u2 * u2).backward()
