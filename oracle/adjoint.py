"""Adjoints of the converged field solve and of the CIC operations (oracle; test infrastructure).

The solve returns u*(delta) with G(u*, delta) = 0 for the discrete Eq. FullDGP2
(see ``oracle.newton``).  Implicit-function theorem: for a loss L(u*),

    J^T mu = dL/du,      dL/ddelta = S^T mu = S mu,

where J = dG/du and S = F^{-1} A (1 - beta/kbar) F acting on delta (its k = 0
multiplier is 0, which also absorbs the mean removal).  H_ij and N are real,
even spectral multipliers, hence self-adjoint, so

    J^T mu = 2 lam (u mu - sum_ij H_ij (h_ij mu)) + alpha mu + gamma N mu.

``adjoint_dense`` solves this with a dense LU (tiny meshes); ``adjoint_picard``
runs the relaxation's own splitting on the transposed system,
mu <- D^{-1} (g + M^T mu), D = 2 (1-w) lam u + alpha, which has the same
iteration spectrum as the forward relaxation linearised at u*.

CIC adjoints differentiate the unquantised weights W = w_x w_y w_z of Eq. CIC;
dw/dx = -N/L for the lower node and +N/L for the upper one.
"""
import numpy as np

from . import spectral as sp
from . import field as fld
from .newton import Operators, _weighted_pair_sum, dense_jacobian
from .pm import _cell_and_weights


def jacobian_t_apply(u, h, mu, ops):
    prm = ops.prm
    hm = {p: h[p] * mu for p in fld.PAIRS}
    tot = 0.0
    for p in fld.PAIRS:
        wgt = 1.0 if p[0] == p[1] else 2.0
        tot = tot + wgt * sp.ifft3(ops.m[p] * sp.fft3(hm[p]), ops.n)
    return 2.0 * prm.lam * (u * mu - tot) + prm.alpha * mu + prm.gamma_eff * ops.nonlocal_(mu)


def source_adjoint(mu, box, prm):
    """S^T mu = S mu: multiplier A (1 - beta/kbar), k = 0 -> 0."""
    n = mu.shape[-1]
    mult = prm.A * (1.0 - prm.beta_eff * sp.inv_kbar(n, box, prm.kappa))
    mult[0, 0, 0] = 0.0
    return sp.ifft3(mult * sp.fft3(mu), n)


def adjoint_dense(u, g, box, prm):
    """mu = J^{-T} g with J assembled densely; returns (mu, dL/ddelta)."""
    n = u.shape[-1]
    ops = Operators(n, box, prm)
    jac = dense_jacobian(u, ops)
    mu = np.linalg.solve(jac.T, np.asarray(g, dtype=np.float64).ravel()).reshape(u.shape)
    return mu, source_adjoint(mu, box, prm)


def adjoint_picard(u, g, box, prm, tol=1e-12, max_iter=200):
    """Transposed relaxation; returns (mu, dL/ddelta, history of <|J^T mu - g|>/<|g|>)."""
    n = u.shape[-1]
    ops = Operators(n, box, prm)
    h = ops.hessian(u)
    g = np.asarray(g, dtype=np.float64)
    gnorm = float(np.mean(np.abs(g)))
    dinv = 1.0 / (2.0 * (1.0 - prm.w) * prm.lam * u + prm.alpha)
    mu = g * dinv
    hist = []
    for _ in range(max_iter):
        res = jacobian_t_apply(u, h, mu, ops) - g
        r = float(np.mean(np.abs(res))) / gnorm
        hist.append(r)
        if r <= tol:
            break
        hm = {p: h[p] * mu for p in fld.PAIRS}
        qsum = 0.0
        for p in fld.PAIRS:
            wgt = 1.0 if p[0] == p[1] else 2.0
            qsum = qsum + wgt * sp.ifft3(ops.m[p] * sp.fft3(hm[p]), n)
        mt_mu = 2.0 * prm.lam * (qsum - prm.w * u * mu) - prm.gamma_eff * ops.nonlocal_(mu)
        mu = dinv * (g + mt_mu)
    return mu, source_adjoint(mu, box, prm), hist


def jvp_solution(u, v_delta, box, prm):
    """du*/ddelta applied to v: J^{-1} S v (dense; tiny meshes), for dot-product tests."""
    n = u.shape[-1]
    ops = Operators(n, box, prm)
    jac = dense_jacobian(u, ops)
    mult = prm.A * (1.0 - prm.beta_eff * sp.inv_kbar(n, box, prm.kappa))
    mult[0, 0, 0] = 0.0
    sv = sp.ifft3(mult * sp.fft3(v_delta), n)
    return np.linalg.solve(jac, sv.ravel()).reshape(u.shape)


def deposit_backward(pos, grad_delta, box):
    """dL/dpos for delta = (N^3/Np) sum_p W(x_p - x_c) - 1 given dL/ddelta on the mesh."""
    g = np.asarray(grad_delta, dtype=np.float64)
    n = g.shape[-1]
    npart = np.asarray(pos).shape[1]
    (i0, i1), (w0, w1) = _cell_and_weights(pos, n, box)
    idx, wts = (i0, i1), (w0, w1)
    dw = (-float(n) / box, float(n) / box)
    out = np.zeros((3, npart))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                gc = g[idx[a][0], idx[b][1], idx[c][2]]
                out[0] += gc * dw[a] * wts[b][1] * wts[c][2]
                out[1] += gc * wts[a][0] * dw[b] * wts[c][2]
                out[2] += gc * wts[a][0] * wts[b][1] * dw[c]
    return out * (float(n) ** 3 / npart)


def interp_backward(mesh, pos, grad_out, box):
    """Adjoint of F_p = sum_c W_c(x_p) F_c: returns (dL/dpos, dL/dmesh)."""
    mesh = np.asarray(mesh, dtype=np.float64)
    go = np.asarray(grad_out, dtype=np.float64)
    m, n = mesh.shape[0], mesh.shape[-1]
    (i0, i1), (w0, w1) = _cell_and_weights(pos, n, box)
    idx, wts = (i0, i1), (w0, w1)
    dw = (-float(n) / box, float(n) / box)
    gpos = np.zeros((3, go.shape[1]))
    gmesh = np.zeros((m, n * n * n))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                flat = (idx[a][0] * n + idx[b][1]) * n + idx[c][2]
                vals = mesh[:, idx[a][0], idx[b][1], idx[c][2]]          # (m, Np)
                proj = np.sum(vals * go, axis=0)
                gpos[0] += proj * dw[a] * wts[b][1] * wts[c][2]
                gpos[1] += proj * wts[a][0] * dw[b] * wts[c][2]
                gpos[2] += proj * wts[a][0] * wts[b][1] * dw[c]
                wgt = wts[a][0] * wts[b][1] * wts[c][2]
                for comp in range(m):
                    np.add.at(gmesh[comp], flat, wgt * go[comp])
    return gpos, gmesh.reshape(m, n, n, n)


def c_power_loss(u, box, prm, target, weights, nbins=64):
    """L = sum_b w_b (P_C,b - P_target,b)^2 with C = lapbar^{-1} u, and dL/du."""
    from .power import power_spectrum, power_spectrum_grad
    c = fld.c_from_u(u, box, prm)
    pk, _, _ = power_spectrum(c, box, nbins)
    diff = pk - target
    loss = float(np.sum(weights * diff * diff))
    dc = power_spectrum_grad(c, 2.0 * weights * diff, box, nbins)
    return loss, fld.c_from_u(dc, box, prm)
