"""GPU (HIP, through the C-ABI) against the CPU oracle on the same seeded inputs.

Tolerances: float64 path <= 1e-10 relative (element-wise comparisons in max norm
where the oracle and the kernels perform the same operations); float32 path
<= 1e-5 relative on the field, 1e-4 on P(k); integer deposit bit-exact.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import field as fld, pm, power, cosmology as cos  # noqa: E402
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
    sys.stdout.flush()


# ---------------------------------------------------------------- FFT
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512])
@pytest.mark.parametrize("prec", [0, 1])
def test_fft_forward_inverse(dgp, n, prec):
    """Forward and inverse 3D transforms against numpy; 256 and 512 run the tile geometries
    chosen for large meshes (one field at 512)."""
    say("fft", n, prec)
    batch = 2 if n <= 256 else 1
    rng = np.random.default_rng(n)
    x = rng.standard_normal((batch, n, n, n))
    ref = np.fft.rfftn(x, axes=(2, 3, 1))        # real transform along axis 0 of each field
    with dgp.Plan(n, 10.0, batch=batch, precision=prec) as plan:
        xs = to_dev(x)
        spec = torch.zeros((batch, n // 2 + 1, n, n), dtype=torch.complex128, device="cuda")
        plan.fft_forward(xs, spec)
        back = torch.zeros_like(xs)
        plan.fft_inverse(spec, back)
        torch.cuda.synchronize()
        got = spec.cpu().numpy()
        tol = 1e-13 if prec == 0 else 3e-6
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)) * np.sqrt(np.log2(n))
        assert np.max(np.abs(back.cpu().numpy() - x)) <= (1e-13 if prec == 0 else 3e-6) * np.max(np.abs(x))


# ---------------------------------------------------------------- field solve, float64
def _c1(n=32, box=64.0, sigma=1.0, seed=1, rnl=3.0):
    delta = inputs.lognormal_delta(n, box, sigma, seed)
    lam = calibrate_lambda(delta, box, rnl)
    return delta, lam


@pytest.mark.parametrize("iters", [0, 1, 3, 7])
def test_solve_same_sequence_fp64(dgp, iters):
    """Exactly `iters` updates from the linear guess: same arithmetic sequence as the oracle."""
    say("solve same-seq", iters)
    n, box = 32, 64.0
    delta, lam = _c1(n, box)
    op = oracle_params(lam=lam)
    u_ref, info_ref = fld.solve(delta, box, op, fixed_iters=iters)
    with dgp.Plan(n, box) as plan:
        p = gpu_params(dgp, lam=lam, tol=0.0, max_iter=iters)
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(p, to_dev(delta), u)
        torch.cuda.synchronize()
        assert info[0]["iters"] == iters
        assert np.max(np.abs(u.cpu().numpy() - u_ref)) <= 1e-12 * np.max(np.abs(u_ref))
        # residual history of the evaluated iterates
        assert abs(info[0]["resid_min"] - min(info_ref.history)) <= 1e-10 * min(info_ref.history) + 1e-15


@pytest.mark.parametrize("n", [8, 16, 64, 128])
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_same_sequence_sizes(dgp, n, prec):
    """Three updates from the linear guess at the mesh sizes the 32^3 case leaves out: each size
    has its own tile shapes, radix plans and Nyquist indices in the axis-2, axis-1 (split Hessian)
    and relaxation kernels.  Float64 to 1e-12 of the oracle; the float32 form to 1e-5."""
    say("solve same-seq sizes", n, prec)
    box = 2.0 * n
    delta, lam = _c1(n, box, seed=40 + n)
    op = oracle_params(lam=lam)
    u_ref, info_ref = fld.solve(delta, box, op, fixed_iters=3)
    with dgp.Plan(n, box, precision=prec) as plan:
        p = gpu_params(dgp, lam=lam, tol=-1.0, max_iter=3)
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(p, to_dev(delta), u)
        torch.cuda.synchronize()
        assert st == 0 and info[0]["iters"] == 3
        if prec == 0:
            assert np.max(np.abs(u.cpu().numpy() - u_ref)) <= 1e-12 * np.max(np.abs(u_ref))
            hist, _ = plan.history()
            assert np.max(np.abs(hist[:3] - np.asarray(info_ref.history[:3])) / np.asarray(info_ref.history[:3])) <= 1e-10
        else:
            assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-5


def test_solve_converged_fp64_c1(dgp):
    """32^3 log-normal (rms 1), screened (r_nl = 3), tolerance 1e-10 (config C1); plus C."""
    say("solve C1")
    n, box = 32, 64.0
    delta, lam = _c1(n, box)
    op = oracle_params(lam=lam, tol=1e-12, max_iter=100)
    u_ref, info_ref = fld.solve(delta, box, op)
    c_ref = fld.c_from_u(u_ref, box, op)
    with dgp.Plan(n, box) as plan:
        p = gpu_params(dgp, lam=lam, tol=1e-12, max_iter=100)
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        c = torch.zeros_like(u)
        st, info = plan.solve_field(p, to_dev(delta), u, c)
        torch.cuda.synchronize()
        assert st == 0 and info[0]["resid"] <= 1e-12
        assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-10
        assert rel_l2(c.cpu().numpy(), c_ref) <= 1e-10
        assert abs(info[0]["eps"] - info_ref.eps) <= 1e-13 * info_ref.eps
        assert abs(info[0]["mean_u"] - info_ref.mean_u) <= 1e-12 * np.max(np.abs(u_ref))
        # the paper's tolerance of 1e-10 on the same input
        p2 = gpu_params(dgp, lam=lam, tol=1e-10, max_iter=100)
        st2, info2 = plan.solve_field(p2, to_dev(delta), u)
        _, i_ref2 = fld.solve(delta, box, op.with_(tol=1e-10))
        assert st2 == 0 and info2[0]["iters"] == i_ref2.iters and info2[0]["resid"] <= 1e-10


def test_solve_warm_zero_init_and_planar(dgp):
    say("solve planar / init modes")
    n, box = 16, 64.0
    x = np.arange(n) * box / n
    delta = 0.8 * np.cos(2 * np.pi * 3 * x / box)[None, :, None] * np.ones((n, n, n))
    op = oracle_params(lam=1.0, tol=1e-13, init=fld.INIT_ZERO)
    u_ref, iref = fld.solve(delta, box, op)
    with dgp.Plan(n, box) as plan:
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=1.0, tol=1e-13, init=dgp.INIT_ZERO), to_dev(delta), u)
        assert st == 0 and info[0]["iters"] == iref.iters
        assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-12
        # warm start from the answer: zero updates
        st, info = plan.solve_field(gpu_params(dgp, lam=1.0, tol=1e-12, init=dgp.INIT_WARM), to_dev(delta), u)
        assert st == 0 and info[0]["iters"] == 0


@pytest.mark.parametrize("init", ["linear", "zero", "warm"])
def test_precision_form_init_modes(dgp, init):
    """The precision form from each initial guess meets the float64 tolerance and lands on
    the oracle's solution; a warm start from the float64 answer needs no float32 pass."""
    say("precision form init", init)
    n, box = 32, 64.0
    delta = inputs.lognormal_delta(n, box, 1.0, 21)
    lam = calibrate_lambda(delta, box, 1.0)
    u_ref, _ = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-12, max_iter=100))
    mode = {"linear": dgp.INIT_LINEAR, "zero": dgp.INIT_ZERO, "warm": dgp.INIT_WARM}[init]
    with dgp.Plan(n, box, precision=dgp.FP32) as plan:
        u = to_dev(u_ref) if init == "warm" else torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-9, max_iter=100, init=mode), to_dev(delta), u)
        assert st == 0 and info[0]["resid"] <= 1e-9
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= 1e-7
        if init == "warm":
            assert info[0]["passes"] - info[0]["passes_fp64"] <= 1


def test_solve_bad_points_same_sequence(dgp):
    """w = 0 at z = 4 on deep voids: bad points, stop at the minimum residual (same decisions)."""
    say("solve bad points")
    n, box = 16, 32.0
    delta = inputs.lognormal_delta(n, box, 1.5, 21)
    op = fld.SolveParams.from_cosmology(OM0, 0.2, tol=1e-12, max_iter=60, lam=1.0, w=0.0, init=fld.INIT_ZERO)
    u_ref, iref = fld.solve(delta, box, op)
    assert iref.status == fld.STATUS_BAD_POINTS
    with dgp.Plan(n, box) as plan:
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        p = dgp.params(OM0, 0.2, lam=1.0, w=0.0, tol=1e-12, max_iter=60, init=dgp.INIT_ZERO)
        st, info = plan.solve_field(p, to_dev(delta), u)
        assert st == 2 and info[0]["status"] == 2
        assert info[0]["iters"] == iref.iters
        assert abs(info[0]["resid"] - iref.resid) <= 1e-9 * iref.resid
        assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_fixed_update_mode(dgp, prec):
    """tol < 0: exactly max_iter updates and the last iterate, the oracle's fixed_iters, also
    through the bad-point regime where the stopping rule would end the solve (w = 0, z = 4)."""
    say("fixed updates", prec)
    n, box = 16, 32.0
    delta = inputs.lognormal_delta(n, box, 1.5, 21)
    k = 9
    op = fld.SolveParams.from_cosmology(OM0, 0.2, lam=1.0, w=0.0, init=fld.INIT_ZERO)
    u_ref, iref = fld.solve(delta, box, op, fixed_iters=k)
    assert max(iref.bad_history) > 0
    with dgp.Plan(n, box, precision=prec) as plan:
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        p = dgp.params(OM0, 0.2, lam=1.0, w=0.0, tol=-1.0, max_iter=k, init=dgp.INIT_ZERO)
        st, info = plan.solve_field(p, to_dev(delta), u)
        assert st == 0 and info[0]["iters"] == k
        if prec == 0:
            hist, bad = plan.history()
            assert np.max(np.abs(hist - np.asarray(iref.history)) / np.asarray(iref.history)) <= 1e-9
            assert np.array_equal(bad[:k], np.asarray(iref.bad_history))
            assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-9
        else:
            assert rel_l2(u.cpu().numpy(), u_ref) <= 1e-4


def test_solve_batched_fp64(dgp):
    """Independent fields in one batched launch; each stops on its own (config C5 shape, smaller mesh)."""
    say("solve batched")
    n, box = 32, 64.0
    sig = [0.3, 1.0, 3.0]
    deltas = np.stack([inputs.lognormal_delta(n, box, s, 500 + i) for i, s in enumerate(sig)])
    lams = [calibrate_lambda(d, box, 3.0) for d in deltas]
    lam = float(np.median(lams))
    with dgp.Plan(n, box, batch=len(sig)) as plan:
        u = torch.zeros(deltas.shape, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-11, max_iter=150), to_dev(deltas), u)
        got = u.cpu().numpy()
    for b in range(len(sig)):
        u_ref, iref = fld.solve(deltas[b], box, oracle_params(lam=lam, tol=1e-11, max_iter=150))
        assert info[b]["status"] == iref.status and info[b]["iters"] == iref.iters
        assert rel_l2(got[b], u_ref) <= 1e-10


# ---------------------------------------------------------------- PM
@pytest.mark.parametrize("fp32", [False, True])
def test_deposit_bit_exact(dgp, fp32):
    say("deposit", fp32)
    n, box = 32, 64.0
    pos, _ = inputs.zeldovich_load(n, box, 11, dtype=np.float32 if fp32 else np.float64)
    grid_ref, delta_ref = pm.deposit(pos, n, box)
    with dgp.Plan(n, box) as plan:
        tdt = torch.float32 if fp32 else torch.float64
        g = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
        d = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.deposit(to_dev(pos, tdt), g, d)
        assert np.array_equal(g.cpu().numpy().reshape(n, n, n), grid_ref)
        assert np.max(np.abs(d.cpu().numpy().reshape(n, n, n) - delta_ref)) <= 1e-14
        perm = np.random.default_rng(1).permutation(pos.shape[1])
        g2 = torch.zeros_like(g)
        plan.deposit(to_dev(pos[:, perm], tdt), g2, None)
        assert torch.equal(g, g2)


def _deposit_cases():
    n, box = 32, 64.0
    rng = np.random.default_rng(5)
    blocked, _ = inputs.zeldovich_load(n, box, 13, block=8)
    shifted = (blocked + 0.49 * box) % box                      # blocks straddle the periodic faces
    uniform = rng.uniform(0.0, box, (3, 5003))                   # boxes exceed the LDS bins: direct path
    cluster = (rng.uniform(-0.7, 0.7, (3, 700)) + box) % box     # one chunk wrapping the corner cell
    mixed = np.concatenate([cluster, uniform[:, :333]], axis=1)  # ragged tail chunk
    tiny = rng.uniform(0.0, box, (3, 37))
    return n, box, {"blocked": blocked, "shifted": shifted, "uniform": uniform, "mixed": mixed, "tiny": tiny}


@pytest.mark.parametrize("case", ["blocked", "shifted", "uniform", "mixed", "tiny"])
def test_deposit_binned_bit_exact(dgp, case):
    """The LDS-binned deposit (compact chunks) and its direct fallback (spread chunks)
    both reproduce the oracle's integer mesh exactly."""
    say("deposit binned", case)
    n, box, cases = _deposit_cases()
    pos = np.ascontiguousarray(cases[case])
    grid_ref, _ = pm.deposit(pos, n, box)
    with dgp.Plan(n, box) as plan:
        g = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
        plan.deposit(to_dev(pos, torch.float64), g, None)
        assert np.array_equal(g.cpu().numpy().reshape(n, n, n), grid_ref)


@pytest.mark.parametrize("fp32", [False, True])
def test_deposit_bit_exact_512(dgp, fp32):
    """From N = 512 the deposit takes wider chunks (2048 particles): its binned path (a compact
    cluster wrapping the corner cell, two full chunks) and its direct fallback (a chunk mixing the
    cluster's tail with spread particles, then a ragged chunk of spread particles) reproduce the
    oracle's integer mesh exactly.  The meshes are compared through their non-zero cells."""
    say("deposit 512", fp32)
    n, box = 512, 1024.0
    rng = np.random.default_rng(17)
    cluster = (rng.uniform(-6.0, 6.0, (3, 5000)) + box) % box
    spread = rng.uniform(0.0, box, (3, 3001))
    pos = np.concatenate([cluster, spread], axis=1)
    pos = np.ascontiguousarray(pos.astype(np.float32) if fp32 else pos)
    ref = pm.cic_deposit_fixed(pos, n, box).reshape(-1)
    ref_idx = np.flatnonzero(ref)
    with dgp.Plan(n, box) as plan:
        g = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
        plan.deposit(to_dev(pos, torch.float32 if fp32 else torch.float64), g, None)
        idx = torch.nonzero(g).reshape(-1)
        vals = g[idx].cpu().numpy()
        idx = idx.cpu().numpy()
        del g
    assert np.array_equal(idx, ref_idx)
    assert np.array_equal(vals, ref[ref_idx])


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_pm_forces(dgp, mode):
    say("forces", mode)
    n, box = 32, 64.0
    pos, _ = inputs.zeldovich_load(n, box, 12)
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 3.0)
    op = oracle_params(lam=lam, tol=1e-12)
    u_ref, _ = fld.solve(delta, box, op)
    f_ref, phik = pm.pm_forces(delta, u_ref, pos, box, op, OM0, 0.5, mode)
    phi_ref = np.fft.irfftn(phik, s=(n, n, n), axes=(0, 1, 2))
    with dgp.Plan(n, box) as plan:
        p = gpu_params(dgp, lam=lam, force_mode=mode)
        force = torch.zeros((3, pos.shape[1]), dtype=torch.float64, device="cuda")
        phi = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.pm_forces(p, to_dev(delta), to_dev(u_ref), to_dev(pos), force, phi)
        assert rel_l2(force.cpu().numpy(), f_ref) <= 1e-10
        assert rel_l2(phi.cpu().numpy().reshape(n, n, n), phi_ref) <= 1e-10


@pytest.mark.parametrize("fp32", [False, True])
def test_step_matches_oracle(dgp, fp32):
    say("step", fp32)
    n, box, a, dlna = 32, 64.0, 0.5, 0.005
    dt = np.float32 if fp32 else np.float64
    pos, psi = inputs.zeldovich_load(n, box, 13, dtype=dt)
    c = cos.coefficients(OM0, a)
    vel = (a * a * c.E * cos.omega_m_of_a(OM0, a) ** 0.55 * psi).astype(dt)
    _, delta = pm.deposit(pos, n, box)
    # r_nl = 1.78 (screened, solvable for this particle load; r_nl >= 3 leaves bad points in its voids)
    lam = calibrate_lambda(delta, box, 1.78)
    op = oracle_params(lam=lam, tol=1e-11)
    x_ref, v_ref, u_ref, info_ref = pm.step(pos, vel, None, a, dlna, box, n, op, OM0)
    with dgp.Plan(n, box) as plan:
        tdt = torch.float32 if fp32 else torch.float64
        tp, tv = to_dev(pos, tdt), to_dev(vel, tdt)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.step(gpu_params(dgp, lam=lam, tol=1e-11), tp, tv, u, dlna)
        assert st == 0 and info["iters"] == info_ref.iters
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= 1e-10
        # displacement of the step (positions themselves carry the lattice offset)
        dx = (tp.cpu().numpy().astype(np.float64) - pos.astype(np.float64) + box / 2) % box - box / 2
        dx_ref = (x_ref.astype(np.float64) - pos.astype(np.float64) + box / 2) % box - box / 2
        tol_x = 1e-10 if not fp32 else 2e-5
        assert rel_l2(dx, dx_ref) <= tol_x
        assert rel_l2(tv.cpu().numpy(), v_ref) <= (1e-12 if not fp32 else 1e-7)


@pytest.mark.parametrize("case", ["blocked", "shifted", "uniform"])
def test_step_particle_orders(dgp, case):
    """Kick-drift with the chunk's force mesh staged in LDS (compact chunks) and the direct
    gather (spread chunks, uniform positions) against the oracle step."""
    say("step order", case)
    n, box, cases = _deposit_cases()
    a, dlna = 0.5, 0.005
    pos = np.ascontiguousarray(cases[case])
    vel = np.random.default_rng(8).normal(0.0, 0.3, pos.shape)
    mode = 0 if case != "uniform" else 2          # uniform positions: GR forces (no field solve)
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 1.78)
    op = oracle_params(lam=lam, tol=1e-11)
    x_ref, v_ref, _, _ = pm.step(pos, vel, None, a, dlna, box, n, op, OM0, mode=mode)
    with dgp.Plan(n, box) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, _ = plan.step(gpu_params(dgp, lam=lam, tol=1e-11, force_mode=mode), tp, tv, u, dlna)
        assert st == 0
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= 1e-10
        assert rel_l2(tv.cpu().numpy() - vel, v_ref - vel) <= 1e-10


def test_step_precision_form(dgp):
    """PM step of a precision-form plan (float32 transforms, float64 polish, float32 force
    mesh) against the float64 oracle step."""
    say("step precision form")
    n, box, a, dlna = 32, 64.0, 0.5, 0.005
    pos, psi = inputs.zeldovich_load(n, box, 13, block=8)
    c = cos.coefficients(OM0, a)
    vel = a * a * c.E * cos.omega_m_of_a(OM0, a) ** 0.55 * psi
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 1.78)
    op = oracle_params(lam=lam, tol=1e-10)
    x_ref, v_ref, u_ref, _ = pm.step(pos, vel, None, a, dlna, box, n, op, OM0)
    with dgp.Plan(n, box, precision=dgp.FP32) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.step(gpu_params(dgp, lam=lam, tol=1e-10), tp, tv, u, dlna)
        assert st == 0 and info["resid"] <= 1e-10
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= 1e-8
        dv = tv.cpu().numpy() - vel
        assert rel_l2(dv, v_ref - vel) <= 1e-5
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= 1e-5


def test_step_bad_point_regime_same_decisions(dgp):
    """r_nl = 10 on a particle load: the relaxation meets bad points in voids and stops at its
    minimum residual (Sec. III C); GPU and oracle take the same decisions (parity of this regime is
    same-sequence agreement only)."""
    say("step r_nl 10")
    n, box = 32, 64.0
    pos, _ = inputs.zeldovich_load(n, box, 13)
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 10.0)
    u_ref, iref = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-11, max_iter=100))
    assert iref.status == fld.STATUS_BAD_POINTS
    with dgp.Plan(n, box) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-11, max_iter=100), to_dev(delta), u)
        assert st == 2 and info[0]["iters"] == iref.iters
        assert abs(info[0]["resid"] - iref.resid) <= 1e-8 * iref.resid
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= 1e-8


def test_power_spectrum(dgp):
    say("power")
    n, box = 32, 64.0
    delta = inputs.lognormal_delta(n, box, 1.0, 3)
    pk_ref, cnt_ref, _ = power.power_spectrum(delta, box)
    op = oracle_params()
    u = fld.linear_solution(fld.source(delta, box, op)[1], box, op)
    pkc_ref, _, _ = power.power_spectrum(fld.c_from_u(u, box, op), box)
    with dgp.Plan(n, box) as plan:
        p = gpu_params(dgp)
        pk, cnt = plan.power_spectrum(p, to_dev(delta))
        assert np.array_equal(cnt, cnt_ref)
        assert np.max(np.abs(pk[0] - pk_ref) / np.where(pk_ref > 0, pk_ref, 1)) <= 1e-12
        pkc, _ = plan.power_spectrum(p, to_dev(u), of_c=True)
        assert np.max(np.abs(pkc[0] - pkc_ref) / np.where(pkc_ref > 0, pkc_ref, 1)) <= 1e-12


# ---------------------------------------------------------------- errors
def test_invalid_arguments(dgp):
    say("errors")
    with pytest.raises(dgp._lib.DGPError):
        dgp.Plan(24, 10.0)
    with pytest.raises(dgp._lib.DGPError):
        dgp.Plan(32, -1.0)
    with dgp.Plan(16, 32.0) as plan:
        d = torch.zeros(16 ** 3, dtype=torch.float64, device="cuda")
        u = torch.zeros_like(d)
        for bad in (dict(lam=float("nan")), dict(w=1.0), dict(lam=-1.0), dict(max_iter=-1)):
            with pytest.raises(dgp._lib.DGPError) as e:
                plan.solve_field(gpu_params(dgp, **bad), d, u)
            assert e.value.code == -1


# ---------------------------------------------------------------- multi-step driver, spherical mode, history
def _run_case():
    n, box = 32, 64.0
    pos, psi = inputs.zeldovich_load(n, box, 17, block=8)
    a0, dlna = 0.45, 0.05
    c = cos.coefficients(OM0, a0)
    vel = a0 * a0 * c.E * cos.omega_m_of_a(OM0, a0) ** 0.55 * psi
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 1.78, a=a0)
    return n, box, pos, vel, a0, dlna, lam


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_run_against_oracle(dgp, prec):
    """dgp_run: one linearised-DGP step before a_switch, three full solves after it (the second
    and third warm-started), against the oracle's driver."""
    say("run", prec)
    n, box, pos, vel, a0, dlna, lam = _run_case()
    x_ref, v_ref, u_ref, infos = pm.run(pos, vel, a0, dlna, 4, 0.47, box, n, OM0, lam, 1e-11)
    assert infos[0] is None and all(i is not None and i.status == 0 for i in infos[1:])
    precision = dgp.FP64 if prec == "fp64" else dgp.FP32
    with dgp.Plan(n, box, precision=precision) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, steps = plan.run(dgp.params(OM0, a0, lam=lam, tol=1e-11, max_iter=100), tp, tv, u, a0, dlna, 4, 0.47)
        assert st == 0 and len(steps) == 4
        assert steps[0]["passes"] == 0 and all(s["resid"] <= 1e-11 for s in steps[1:])
        if prec == "fp64":   # same decisions as the oracle, warm starts included
            assert [s["iters"] for s in steps[1:]] == [i.iters for i in infos[1:]]
        tol = 1e-9 if prec == "fp64" else 1e-5
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= (1e-9 if prec == "fp64" else 1e-8)
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= tol
        assert rel_l2(tv.cpu().numpy() - vel, v_ref - vel) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_run_resumes_from_saved_state(dgp, prec):
    """A run's state is (positions, velocities, u_state, a): four steps in one call equal two
    steps, a copy of the state, and two more steps resumed from the copy with a warm start (in a
    fresh plan, so no plan-held state carries over), up to the rounding of the scale factor (the
    resumed run forms a = a_2 e^(k dlna) where the whole run forms a_0 e^((k+2) dlna)) and the
    solve tolerance."""
    say("run resume", prec)
    n, box, pos, vel, a0, dlna, lam = _run_case()
    precision = dgp.FP64 if prec == "fp64" else dgp.FP32
    prm = dgp.params(OM0, a0, lam=lam, tol=1e-11, max_iter=100)
    with dgp.Plan(n, box, precision=precision) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, _ = plan.run(prm, tp, tv, u, a0, dlna, 4, 0.47)
        assert st == 0
        whole = [x.cpu().numpy() for x in (tp, tv, u)]
    with dgp.Plan(n, box, precision=precision) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, _ = plan.run(prm, tp, tv, u, a0, dlna, 2, 0.47)
        assert st == 0
        saved = [x.cpu().numpy().copy() for x in (tp, tv, u)]
    with dgp.Plan(n, box, precision=precision) as plan:
        tp, tv, u = (to_dev(x) for x in saved)
        u = u.reshape(-1).contiguous()
        a2 = a0 * np.exp(2 * dlna)
        st, _ = plan.run(dgp.params(OM0, a2, lam=lam, tol=1e-11, max_iter=100, init=dgp.INIT_WARM), tp, tv, u, a2,
                         dlna, 2, 0.47)
        assert st == 0
        resumed = [x.cpu().numpy() for x in (tp, tv, u)]
    dx_w = (whole[0] - pos + box / 2) % box - box / 2
    dx_r = (resumed[0] - pos + box / 2) % box - box / 2
    assert rel_l2(dx_r, dx_w) <= 1e-10
    assert rel_l2(resumed[1] - vel, whole[1] - vel) <= 1e-10
    assert rel_l2(resumed[2].reshape(-1), whole[2].reshape(-1)) <= 1e-9


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_comparison_runs_against_oracle(dgp, mode):
    """The lDGP, GRH and GR comparison runs (Sec. IV): dgp_run with that force law at every step
    (GR in its own LCDM background, kick-drift included) against the oracle's driver."""
    say("comparison run", mode)
    n, box, pos, vel, a0, dlna, lam = _run_case()
    x_ref, v_ref, _, infos = pm.run(pos, vel, a0, dlna, 3, 0.47, box, n, OM0, lam, 1e-11, mode=mode)
    with dgp.Plan(n, box) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, steps = plan.run(dgp.params(OM0, a0, lam=lam, tol=1e-11, max_iter=100, force_mode=mode), tp, tv, u, a0,
                             dlna, 3, 0.47)
        assert st == 0 and all(s["passes"] == 0 for s in steps)
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= 1e-10
        assert rel_l2(tv.cpu().numpy() - vel, v_ref - vel) <= 1e-10


@pytest.mark.parametrize("w", [0.0, 0.25, 1.0 / 3.0, 0.5, 0.8])
def test_w_scan_fig3(dgp, w):
    """The w-scan of Sec. III C (Fig. 3) on the z = 24 particle density of the oracle's Fig. 3 test
    (lam = 1, the same linear solution for every w, 20 updates): residual and bad-fraction history
    of every update against the oracle, including the w = 0 run through its bad points."""
    say("w scan", w)
    from tests.test_oracle_pins import _fig3_delta
    delta = _fig3_delta()
    n, box, k = 64, 16.0, 20
    prm = fld.SolveParams.from_cosmology(OM0, 1 / 25, lam=1.0, w=w)
    u_ref, iref = fld.solve(delta, box, prm, fixed_iters=k)
    with dgp.Plan(n, box) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(dgp.params(OM0, 1 / 25, lam=1.0, w=w, tol=-1.0, max_iter=k), to_dev(delta), u)
        assert st == 0 and info[0]["iters"] == k
        hist, bad = plan.history()
        href = np.asarray(iref.history)
        assert len(hist) == k + 1
        # relative, down to an absolute floor: r near 1e-10 is a mean of float64 cancellations
        assert np.all(np.abs(hist - href) <= (1e-9 if w > 0 else 1e-7) * href + 1e-14)
        assert np.array_equal(bad[:k] * n ** 3, np.asarray(iref.bad_history) * n ** 3)
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= (1e-10 if w > 0 else 1e-7)


def test_spherical_mode(dgp):
    """spherical = 1: the first w = 1/3 update from zero (Eq. SphPoi) for a solve, and the
    spherical-mode PM run, against the oracle."""
    say("spherical")
    n, box = 32, 64.0
    delta = inputs.lognormal_delta(n, box, 1.0, 23)
    lam = calibrate_lambda(delta, box, 3.0)
    op = oracle_params(lam=lam)
    u_ref = fld.spherical_first_update(delta, box, op)
    with dgp.Plan(n, box) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, spherical=1), to_dev(delta), u)
        assert st == 0 and info[0]["iters"] == 1 and info[0]["passes"] == 0 and info[0]["resid"] == -1.0
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= 1e-13
        assert abs(info[0]["mean_u"] - u_ref.mean()) <= 1e-12 * np.max(np.abs(u_ref))
    n, box, pos, vel, a0, dlna, lam = _run_case()
    x_ref, v_ref, _, _ = pm.run(pos, vel, a0, dlna, 2, 0.0, box, n, OM0, lam, 1e-11, spherical=True)
    with dgp.Plan(n, box) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, _ = plan.run(dgp.params(OM0, a0, lam=lam, spherical=1), tp, tv, u, a0, dlna, 2, 0.0)
        assert st == 0
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= 1e-10


def test_solve_history(dgp):
    """Residual and bad-fraction history per pass (Fig. 3 quantities): the w = 1/3 solve
    contracts monotonically with no bad points; w = 0 on deep voids meets bad points."""
    say("history")
    n, box = 16, 32.0
    delta = inputs.lognormal_delta(n, box, 1.0, 5)
    lam = calibrate_lambda(delta, box, 1.0)
    with dgp.Plan(n, box) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-10, max_iter=100), to_dev(delta), u)
        r, bad = plan.history()
        assert st == 0 and len(r) == info[0]["passes"] == info[0]["iters"] + 1
        assert r[-1] == info[0]["resid"] and np.all(np.diff(r) < 0) and np.all(bad == 0)
        _, i_ref = fld.solve(delta, box, oracle_params(lam=lam, tol=1e-10, max_iter=100))
        assert abs(r[-1] - i_ref.resid) <= 1e-6 * i_ref.resid
    n, box = 16, 32.0
    delta = inputs.lognormal_delta(n, box, 1.5, 21)   # the bad-point case of the same-sequence test
    with dgp.Plan(n, box) as plan:
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        p = dgp.params(OM0, 0.2, lam=1.0, w=0.0, tol=1e-12, max_iter=60, init=dgp.INIT_ZERO)
        st, info = plan.solve_field(p, to_dev(delta), u)
        r, bad = plan.history()
        assert st == 2 and np.max(bad) > 0 and len(r) == info[0]["passes"]
