"""Independent Newton solvers of the same discrete equation (oracle; test infrastructure).

The relaxation of Sec. III B/C is an iteration whose fixed point is the exact
solution of the discrete Eq. FullDGP2,

    G(u) = lam [u^2 - sum_ij (H_ij u)^2] + alpha u + gamma N u - S = 0,

with H_ij and N the spectral multipliers of ``oracle.spectral``.  This module
finds that root by Newton's method instead (no w-split, no quadratic formula),
so agreement of the two fixed points pins the relaxation's update, branch choice
and stopping rule.  Newton-Krylov (GMRES on the Jacobian action) is used for
N >= 16; a dense Newton with the Jacobian assembled column by column for tiny N.
The physical branch is selected by starting from the linear solution, to which
the root reduces as lam -> 0 (Sec. III B).
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, gmres

from . import spectral as sp
from .field import source, linear_solution, PAIRS


class Operators:
    """H_ij and N as spectral multipliers on an n^3 mesh."""

    def __init__(self, n, box, prm):
        self.n = n
        self.m = {p: sp.hessian_multiplier(p[0], p[1], n, box) for p in PAIRS}
        self.minus_inv_kbar = -sp.inv_kbar(n, box, prm.kappa)
        self.prm = prm

    def hessian(self, v):
        vk = sp.fft3(v)
        return {p: sp.ifft3(self.m[p] * vk, self.n) for p in PAIRS}

    def nonlocal_(self, v):
        if not self.prm.nonlocal_terms:
            return np.zeros_like(v)
        return sp.ifft3(self.minus_inv_kbar * sp.fft3(v), self.n)


def _weighted_pair_sum(a, b):
    """sum over all (i, j) of a_ij b_ij with a, b given on the 6 independent pairs."""
    tot = 0.0
    for p in PAIRS:
        wgt = 1.0 if p[0] == p[1] else 2.0
        tot = tot + wgt * a[p] * b[p]
    return tot


def g_of_u(u, s, ops):
    prm = ops.prm
    h = ops.hessian(u)
    return prm.lam * (u * u - _weighted_pair_sum(h, h)) + prm.alpha * u + prm.gamma_eff * ops.nonlocal_(u) - s


def jacobian_apply(u, h, v, ops):
    """J v = 2 lam (u v - sum_ij h_ij H_ij v) + alpha v + gamma N v."""
    prm = ops.prm
    hv = ops.hessian(v)
    return 2.0 * prm.lam * (u * v - _weighted_pair_sum(h, hv)) + prm.alpha * v + prm.gamma_eff * ops.nonlocal_(v)


def newton_krylov(delta, box, prm, tol=1e-13, max_newton=30, u0=None):
    """Newton with GMRES inner solves.  Returns (u, history of max|G|/eps)."""
    n = delta.shape[-1]
    s, sk, eps = source(delta, box, prm)
    ops = Operators(n, box, prm)
    u = linear_solution(sk, box, prm) if u0 is None else np.array(u0, dtype=np.float64)
    hist = []
    for _ in range(max_newton):
        g = g_of_u(u, s, ops)
        r = float(np.mean(np.abs(g)) / eps)
        hist.append(r)
        if r <= tol:
            break
        h = ops.hessian(u)
        size = u.size
        op = LinearOperator((size, size), dtype=np.float64,
                            matvec=lambda x: jacobian_apply(u, h, x.reshape(u.shape), ops).ravel())
        du, _ = gmres(op, -g.ravel(), rtol=1e-14, atol=0.0, restart=200, maxiter=20)
        u = u + du.reshape(u.shape)
    return u, hist


def dense_jacobian(u, ops):
    """J assembled column by column (J e_x for every unit vector e_x); tiny meshes only."""
    size = u.size
    h = ops.hessian(u)
    jac = np.empty((size, size))
    e = np.zeros(size)
    for col in range(size):
        e[col] = 1.0
        jac[:, col] = jacobian_apply(u, h, e.reshape(u.shape), ops).ravel()
        e[col] = 0.0
    return jac


def dense_newton(delta, box, prm, tol=1e-14, max_newton=30):
    """Newton with a dense direct solve at every step (tiny meshes only)."""
    n = delta.shape[-1]
    s, sk, eps = source(delta, box, prm)
    ops = Operators(n, box, prm)
    u = linear_solution(sk, box, prm)
    hist = []
    for _ in range(max_newton):
        g = g_of_u(u, s, ops)
        r = float(np.mean(np.abs(g)) / eps)
        hist.append(r)
        if r <= tol:
            break
        jac = dense_jacobian(u, ops)
        u = u - np.linalg.solve(jac, g.ravel()).reshape(u.shape)
    return u, hist
