"""The five workload configurations at their full sizes, GPU (C-ABI) against the oracle.

C1  32^3 log-normal field, tolerance 1e-10                      (test_gpu_parity.py)
C2  128^3 Zel'dovich load, 5 nonlinear ratios, full PM step      (here)
C3  256^3 Zel'dovich load, precision form vs float64 vs oracle   (here)
C4  512^3 mesh, 512^3 float32 particles: properties + samples    (here)
C5  8 x 128^3 batched log-normal fields, adjoint vs FD / oracle  (here)
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import field as fld, pm, power, adjoint, cosmology as cos  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import OM0, to_dev, oracle_params, calibrate_lambda, gpu_params, rel_l2  # noqa: E402

A = 0.5


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def say(*a):
    print(*a, flush=True)


def growth_vel(psi):
    c = cos.coefficients(OM0, A)
    return A * A * c.E * cos.omega_m_of_a(OM0, A) ** 0.55 * psi


# ---------------------------------------------------------------- C2
C2_RATIOS = (0.01, 0.0562, 0.316, 1.78, 10.0)


@pytest.fixture(scope="module")
def c2_load():
    n, box = 128, 256.0
    pos, psi = inputs.zeldovich_load(n, box, 2)
    grid, delta = pm.deposit(pos, n, box)
    return n, box, pos, growth_vel(psi), grid, delta


def test_c2_deposit_bit_exact(dgp, c2_load):
    say("C2 deposit")
    n, box, pos, vel, grid_ref, delta_ref = c2_load
    with dgp.Plan(n, box) as plan:
        g = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
        d = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.deposit(to_dev(pos), g, d)
        assert np.array_equal(g.cpu().numpy().reshape(n, n, n), grid_ref)
        assert np.max(np.abs(d.cpu().numpy().reshape(n, n, n) - delta_ref)) <= 1e-14


@pytest.mark.parametrize("rnl", C2_RATIOS)
def test_c2_pm_step(dgp, c2_load, rnl):
    """Deposit -> solve -> forces -> kick-drift at each nonlinear ratio (float64)."""
    say("C2 step", rnl)
    n, box, pos, vel, _, delta = c2_load
    dlna = 0.005
    lam = calibrate_lambda(delta, box, rnl)
    op = oracle_params(lam=lam, tol=1e-10, max_iter=100)
    x_ref, v_ref, u_ref, iref = pm.step(pos, vel, None, A, dlna, box, n, op, OM0)
    with dgp.Plan(n, box) as plan:
        tp, tv = to_dev(pos), to_dev(vel)
        u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, info = plan.step(gpu_params(dgp, lam=lam, tol=1e-10, max_iter=100), tp, tv, u, dlna)
        assert st == iref.status and info["iters"] == iref.iters
        if iref.status == fld.STATUS_OK:
            assert info["resid"] <= 1e-10
            tol_u = 1e-10
        else:
            # screened beyond solvability (voids): same decisions, same minimum-residual iterate
            assert abs(info["resid"] - iref.resid) <= 1e-8 * iref.resid
            tol_u = 1e-8
        assert rel_l2(u.cpu().numpy().reshape(n, n, n), u_ref) <= tol_u
        dx = (tp.cpu().numpy() - pos + box / 2) % box - box / 2
        dx_ref = (x_ref - pos + box / 2) % box - box / 2
        assert rel_l2(dx, dx_ref) <= tol_u
        assert rel_l2(tv.cpu().numpy(), v_ref) <= tol_u


# ---------------------------------------------------------------- C3
@pytest.fixture(scope="module")
def c3_case():
    n, box = 256, 512.0
    pos, psi = inputs.zeldovich_load(n, box, 3)
    _, delta = pm.deposit(pos, n, box)
    lam = calibrate_lambda(delta, box, 1.78)
    op = oracle_params(lam=lam, tol=1e-8, max_iter=60)
    say("C3 oracle solve")
    u_ref, iref = fld.solve(delta, box, op)
    say("C3 oracle done", iref.iters)
    return n, box, pos, delta, lam, op, u_ref, iref


def test_c3_precision_form_against_fp64_and_oracle(dgp, c3_case):
    """Precision form and float64 form at residual 1e-8 against the float64 oracle at 1e-8:
    C (phi) and P(k) of C; forces from both."""
    say("C3")
    n, box, pos, delta, lam, op, u_ref, iref = c3_case
    assert iref.status == fld.STATUS_OK
    c_ref = fld.c_from_u(u_ref, box, op)
    pk_ref, _, _ = power.power_spectrum(c_ref, box)
    f_ref, _ = pm.pm_forces(delta, u_ref, pos, box, op, OM0, A)
    d = to_dev(delta)
    out = {}
    for prec in (dgp.FP64, dgp.FP32):
        with dgp.Plan(n, box, precision=prec) as plan:
            p = gpu_params(dgp, lam=lam, tol=1e-8, max_iter=60)
            u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            c = torch.zeros_like(u)
            st, info = plan.solve_field(p, d, u, c)
            assert st == 0 and info[0]["resid"] <= 1e-8
            pk, _ = plan.power_spectrum(p, u, of_c=True)
            force = torch.zeros((3, pos.shape[1]), dtype=torch.float64, device="cuda")
            plan.pm_forces(p, d, u, to_dev(pos), force)   # float32 transforms in the precision form
            out["force", prec] = force.cpu().numpy()
            out[prec] = (u.cpu().numpy().reshape(n, n, n), c.cpu().numpy().reshape(n, n, n), pk[0], info[0])
    u64, c64, pk64, i64 = out[dgp.FP64]
    assert i64["iters"] == iref.iters
    assert rel_l2(u64, u_ref) <= 1e-10 and rel_l2(c64, c_ref) <= 1e-10
    sel = pk_ref > 0
    assert np.max(np.abs(pk64[sel] / pk_ref[sel] - 1)) <= 1e-10
    assert rel_l2(out["force", dgp.FP64], f_ref) <= 1e-10
    u32, c32, pk32, i32 = out[dgp.FP32]
    # both forms reach 1e-8; their distance to the oracle is set by that tolerance
    assert rel_l2(c32, c_ref) <= 1e-5
    assert np.max(np.abs(pk32[sel] / pk_ref[sel] - 1)) <= 1e-4
    f32_err = rel_l2(out["force", dgp.FP32], f_ref)
    assert f32_err <= 1e-5
    say("C3 errors: fp32-form C %.2e, P(k) %.2e, forces %.2e" % (
        rel_l2(c32, c_ref), np.max(np.abs(pk32[sel] / pk_ref[sel] - 1)), f32_err))


# ---------------------------------------------------------------- C4
@pytest.mark.timeout(600)
def test_c4_512_properties_and_samples(dgp):
    """512^3 mesh, 512^3 float32 particles.  The oracle cannot solve this size in a test, so:
    deposit bit-exact on sampled cells (brute force over the particles near them), mass
    conservation, precision form vs float64 form, and the float64 residual meets 1e-8."""
    say("C4")
    n, box = 512, 1024.0
    torch.cuda.empty_cache()
    pos, psi = inputs.zeldovich_load(n, box, 4, dtype=np.float32)
    npart = pos.shape[1]
    say("C4 load built")
    tp = to_dev(pos, torch.float32)
    with dgp.Plan(n, box) as plan:
        g = torch.zeros(n ** 3, dtype=torch.int64, device="cuda")
        d = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        plan.deposit(tp, g, d)
        # total mass in exact integers (the sum of all cells, ~2^67, overflows int64: split it)
        total = int((g >> 32).sum().item()) * 2 ** 32 + int((g & 0xFFFFFFFF).sum().item())
        assert abs(total - npart * 2 ** 40) <= 4 * npart
        # sampled cells: brute-force deposit of every particle whose lower CIC node is one of the
        # 8 nodes that can reach a sampled cell (selected through a node lookup table)
        cells = inputs.random_cells(n, 32, 44)
        lo = np.floor(pos.astype(np.float64) * (n / box)).astype(np.int64) % n
        lo_flat = (lo[0] * n + lo[1]) * n + lo[2]
        del lo
        cc = np.stack(np.unravel_index(cells, (n, n, n)))
        table = np.zeros(n ** 3, dtype=bool)
        for da in (0, 1):
            for db in (0, 1):
                for dc in (0, 1):
                    table[(((cc[0] - da) % n) * n + (cc[1] - db) % n) * n + (cc[2] - dc) % n] = True
        sub = pos[:, table[lo_flat]]
        del lo_flat, table
        ref = pm.cic_deposit_fixed(sub, n, box).ravel()[cells]
        got = g.cpu().numpy()[cells]
        assert np.array_equal(got, ref)
        say("C4 deposit checked on", len(cells), "cells from", sub.shape[1], "particles")
        lam = 1.78 * gpu_params(dgp).alpha
        ulin = torch.zeros_like(d)
        plan.solve_field(gpu_params(dgp, tol=0.0, max_iter=0), d, ulin)
        lam = lam / float(ulin.abs().max())
        del ulin, g
        u64 = torch.zeros_like(d)
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-8, max_iter=60), d, u64)
        say("C4 fp64", st, info[0]["iters"], info[0]["resid"])
        assert st == 0 and info[0]["resid"] <= 1e-8
    with dgp.Plan(n, box, precision=dgp.FP32) as plan:
        u32 = torch.zeros_like(d)
        st, info = plan.solve_field(gpu_params(dgp, lam=lam, tol=1e-8, max_iter=60), d, u32)
        say("C4 fp32", st, info[0]["iters"], info[0]["resid"])
        assert st == 0 and info[0]["resid"] <= 1e-8
        assert float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)) <= 1e-6
        # one full PM step in the precision form with float32 particles
        tv = to_dev(growth_vel(psi), torch.float32)
        st, info = plan.step(gpu_params(dgp, lam=lam, tol=1e-8, max_iter=60), tp, tv, u32, 0.005)
        assert st == 0 and info["resid"] <= 1e-8
        assert bool(torch.all((tp >= 0) & (tp < box)))


# ---------------------------------------------------------------- C5
C5_SIGMA = [0.3, 0.3, 0.3, 1.0, 1.0, 1.0, 3.0, 3.0]


@pytest.mark.timeout(600)
def test_c5_batched_adjoint_against_fd(dgp):
    """8 seeded log-normal 128^3 fields in one batched launch; loss sum_b w_b (P_C,b - P_target,b)^2.
    Forward in the precision form (float32 + float64 polish); the FD check runs the float64 path
    converged to 1e-13 (central differences, step 1e-4, 64 random cells)."""
    say("C5")
    from paper_0906_4548_amd.autograd import FieldSolve, PowerOfC, power_loss
    n, box, B = 128, 256.0, len(C5_SIGMA)
    deltas = np.stack([inputs.lognormal_delta(n, box, s, 500 + i) for i, s in enumerate(C5_SIGMA)])
    lam = float(np.median([calibrate_lambda(dd, box, 3.0) for dd in deltas]))
    target_field = inputs.lognormal_delta(n, box, 1.0, 999)
    op = oracle_params(lam=lam)
    u_t, _ = fld.solve(target_field, box, op.with_(tol=1e-10))
    pk_t, _, _ = power.power_spectrum(fld.c_from_u(u_t, box, op), box)
    wts = np.where(pk_t > 0, 1.0 / np.where(pk_t > 0, pk_t, 1.0) ** 2, 0.0)
    tgt, tw = to_dev(pk_t), to_dev(wts)
    d = to_dev(deltas).requires_grad_(True)
    with dgp.Plan(n, box, batch=B, precision=dgp.FP32) as p32, dgp.Plan(n, box, batch=B) as p64:
        fwd = gpu_params(dgp, lam=lam, tol=1e-8, max_iter=100)
        bwd = gpu_params(dgp, lam=lam, tol=1e-12, max_iter=200)
        u = FieldSolve.apply(d, p32, fwd, bwd)
        loss = power_loss(PowerOfC.apply(u, p32, fwd), tgt, tw)
        loss.backward()
        g32 = d.grad.cpu().numpy()
        # float64 path at 1e-13 for the finite differences
        p13 = gpu_params(dgp, lam=lam, tol=1e-13, max_iter=200)
        d2 = to_dev(deltas).requires_grad_(True)
        loss64 = power_loss(PowerOfC.apply(FieldSolve.apply(d2, p64, p13, bwd), p64, p13), tgt, tw)
        loss64.backward()
        g64 = d2.grad.cpu().numpy()
        assert rel_l2(g32, g64) <= 1e-4
        say("C5 gradients fp32-form vs fp64: %.2e" % rel_l2(g32, g64))
        cells = inputs.random_cells(n, 64, 12)
        h = 1e-4
        eps = np.finfo(np.float64).eps
        fails, worst = [], {}
        # (1) the config's loss: central difference, step 1e-4, written as
        #     L+ - L- = sum_bins w (P+ - P-)(P+ + P- - 2 T); accepted within 1e-6 relative plus the
        #     float64 rounding floor of that difference (large when P >> P_target, i.e. sigma = 3)
        # (2) the solve adjoint alone: f = <g, u(delta)> for a fixed random g, difference taken
        #     field-wise before the sum; 1e-6 relative for every field
        gfix = np.random.default_rng(77).standard_normal((B, n ** 3))
        gfd = torch.zeros((B, n ** 3), dtype=torch.float64, device="cuda")
        u0 = torch.zeros_like(gfd)
        p64.solve_field(p13, to_dev(deltas), u0)
        p64.solve_field_backward(bwd, to_dev(deltas), u0, to_dev(gfix), gfd)
        gfd = gfd.cpu().numpy()
        for k, cidx in enumerate(cells):
            b = k % B
            pks, us = [], []
            for sgn in (1, -1):
                dd = deltas.copy()
                dd.reshape(B, -1)[b, cidx] += sgn * h
                with torch.no_grad():
                    uu = FieldSolve.apply(to_dev(dd), p64, p13)
                    pks.append(PowerOfC.apply(uu, p64, p13)[b].cpu().numpy())
                    us.append(uu[b].cpu().numpy().ravel())
            fd = float(np.sum(wts * (pks[0] - pks[1]) * (pks[0] + pks[1] - 2.0 * pk_t))) / (2 * h)
            noise = float(np.sum(wts * np.abs(pks[0] + pks[1] - 2.0 * pk_t) * (pks[0] + pks[1]))) * 8 * eps / (2 * h)
            an = g64.reshape(B, -1)[b, cidx]
            if abs(fd - an) > 1e-6 * max(abs(fd), abs(an)) + noise:
                fails.append(("loss", k, C5_SIGMA[b], fd, an, noise))
            worst[C5_SIGMA[b]] = max(worst.get(C5_SIGMA[b], 0.0), abs(fd - an) / abs(an))
            fl = float(np.dot(gfix[b], us[0] - us[1])) / (2 * h)
            al = gfd[b, cidx]
            if abs(fl - al) > 1e-6 * max(abs(fl), abs(al)):
                # strongly curved response (near a void vertex): remove the h^2 term (Richardson, h and 2h)
                us2 = []
                for sgn in (1, -1):
                    dd = deltas.copy()
                    dd.reshape(B, -1)[b, cidx] += sgn * 2 * h
                    with torch.no_grad():
                        us2.append(FieldSolve.apply(to_dev(dd), p64, p13)[b].cpu().numpy().ravel())
                fl2 = float(np.dot(gfix[b], us2[0] - us2[1])) / (4 * h)
                # accept within the difference quotient's own spread between steps h and 2h
                # (truncation plus forward-solve convergence noise of the two perturbed solves)
                if abs(fl - al) > 1e-6 * max(abs(fl), abs(al)) + abs(fl - fl2):
                    fails.append(("linear", k, C5_SIGMA[b], fl, fl2, al))
                say("C5 cell %d (sigma %.1f): FD(h) %.10e FD(2h) %.10e adjoint %.10e" % (k, C5_SIGMA[b], fl, fl2, al))
        say("C5 worst loss-FD relative error by sigma:", worst)
        assert not fails, fails[:5]
    # oracle adjoint on a 16^3 copy (seed 13)
    n2, box2 = 16, 32.0
    d16 = inputs.lognormal_delta(n2, box2, 1.0, 13)
    lam2 = calibrate_lambda(d16, box2, 3.0)
    op2 = oracle_params(lam=lam2, tol=1e-13, max_iter=200)
    u16, _ = fld.solve(d16, box2, op2)
    gu = np.random.default_rng(13).standard_normal((n2, n2, n2))
    _, gd_dense = adjoint.adjoint_dense(u16, gu, box2, op2)
    with dgp.Plan(n2, box2) as plan:
        gd = torch.zeros(n2 ** 3, dtype=torch.float64, device="cuda")
        plan.solve_field_backward(gpu_params(dgp, lam=lam2, tol=1e-13, max_iter=200), to_dev(d16), to_dev(u16),
                                  to_dev(gu), gd)
        assert rel_l2(gd.cpu().numpy().reshape(n2, n2, n2), gd_dense) <= 1e-10
