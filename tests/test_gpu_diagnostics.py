"""GPU diagnostics (non-elliptic fraction, P_c/P_m, Delta_gradC) against the CPU oracle.

The fraction is an integer count over the mesh: it must agree exactly except at points whose
ellipticity matrix has an eigenvalue within rounding of zero (the oracle reports the smallest
|eigenvalue| per point; the kernel decides by Sylvester's criterion on float64 minors).
Spectra: float64, <= 1e-12 relative per bin.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diagnostics, field as fld  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import OM0, to_dev, oracle_params, calibrate_lambda, gpu_params  # noqa: E402


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


def _allowed(u, box, op):
    """Oracle fraction and the number of points whose decision is within rounding."""
    frac, min_ev = diagnostics.nonelliptic_fraction(u, box, op)
    scale = np.max(np.abs(op.alpha) + 2 * abs(op.lam) * np.abs(u))
    return frac, int(np.count_nonzero(min_ev <= 1e-10 * scale))


def test_nonelliptic_plane_wave(dgp):
    """u = A cos(2 pi x / L) with alpha / (2 lam A) = 1/2: a third of the points is not elliptic."""
    say("diag plane wave")
    n, box, a = 32, 64.0, 0.5
    op = oracle_params(a, lam=1.0)
    amp = op.alpha / op.lam
    x = (np.arange(n) + 0.25) * box / n
    u = amp * np.cos(2.0 * np.pi * x / box)[:, None, None] * np.ones((n, n, n))
    ref, near = _allowed(u, box, op)
    assert near == 0
    with dgp.Plan(n, box) as plan:
        ne, ratio, dgc = plan.diagnostics(gpu_params(dgp, a, lam=1.0), None, to_dev(u))
    assert ratio is None
    assert ne[0] == ref
    assert abs(ref - 1.0 / 3.0) <= 1.0 / n


@pytest.mark.parametrize("n", [16, 32])
def test_nonelliptic_fraction_batch(dgp, n):
    """Two linear-theory fields as test inputs: one mirrored (u -> -u, so that the peaks cross
    2 lam u + alpha = 0: a few isolated non-elliptic points) and one scaled tenfold (most points
    non-elliptic)."""
    say("diag nonelliptic", n)
    box, a = 2.0 * n, 0.5
    delta = inputs.lognormal_delta(n, box, 1.0, 3)
    lam = calibrate_lambda(delta, box, 3.0, a)
    op = oracle_params(a, lam=lam)
    us = []
    for seed, scale in ((3, -1.0), (4, 10.0)):
        d = inputs.lognormal_delta(n, box, 1.0, seed)
        us.append(scale * fld.linear_solution(fld.source(d, box, op)[1], box, op))
    refs = [_allowed(u, box, op) for u in us]
    assert 0.0 < refs[0][0] < 0.05 and 0.5 < refs[1][0] < 1.0
    with dgp.Plan(n, box, batch=2) as plan:
        ne, _, _ = plan.diagnostics(gpu_params(dgp, a, lam=lam), None, to_dev(np.stack(us)))
    for b in range(2):
        ref, near = refs[b]
        assert abs(ne[b] - ref) * n ** 3 <= near + 1e-9, (b, ne[b], ref, near)


def test_spectra_diagnostics(dgp):
    """P_c/P_m (Eq. cdef) and Delta_gradC (Eq. DGradC) of solved fields, batch of two."""
    say("diag spectra")
    n, box, a, nbins = 32, 64.0, 0.5, 24
    deltas = [inputs.lognormal_delta(n, box, 1.0, s) for s in (11, 12)]
    lam = calibrate_lambda(deltas[0], box, 2.0, a)
    op = oracle_params(a, lam=lam, tol=1e-11, max_iter=200)
    us = [fld.solve(d, box, op)[0] for d in deltas]
    with dgp.Plan(n, box, batch=2) as plan:
        ne, ratio, dgc = plan.diagnostics(gpu_params(dgp, a, lam=lam), to_dev(np.stack(deltas)),
                                          to_dev(np.stack(us)), nbins=nbins)
    for b in range(2):
        r_ref = diagnostics.pc_over_pm(deltas[b], us[b], box, OM0, a, nbins)
        g_ref = diagnostics.delta_gradc(us[b], box, op, nbins)
        assert np.max(np.abs(ratio[b] - r_ref)) <= 1e-12 * np.max(np.abs(r_ref))
        assert np.max(np.abs(dgc[b] - g_ref)) <= 1e-12 * np.max(np.abs(g_ref))
        ref, near = _allowed(us[b], box, op)
        assert abs(ne[b] - ref) * n ** 3 <= near + 1e-9


def test_diagnostics_errors(dgp):
    """Argument errors come back as DGP_E_INVALID (no GPU work is issued for them)."""
    say("diag errors")
    n, box = 16, 32.0
    u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    with dgp.Plan(n, box) as plan:
        prm = gpu_params(dgp)
        for nb in (0, 129):
            with pytest.raises(dgp._lib.DGPError):
                plan.diagnostics(prm, u, u, nbins=nb)
        # P_c/P_m needs delta: the C entry point rejects it (the binding passes NULL for None and
        # then asks for no ratio, so call the entry point directly)
        import ctypes
        ratio = np.zeros(8)
        rc = dgp._lib.load().dgp_diagnostics(plan.handle, ctypes.byref(prm), None,
                                              ctypes.c_void_p(u.data_ptr()), None,
                                              ratio.ctypes.data_as(ctypes.c_void_p), None, 8, None)
        assert rc == -1
        ne, ratio_none, dgc = plan.diagnostics(prm, None, u, nbins=8)
        assert ratio_none is None and ne[0] == 0.0
