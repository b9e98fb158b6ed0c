"""Particle-mesh step around the field solve (oracle; test infrastructure).

Follows Sec. III A "PM N-body Simulations": CIC mass assignment (Eq. CIC),
the modified Poisson equation (Eq. FullDGP1) solved in Fourier space, the
spectral gradient i k phi, CIC interpolation of the force with the same
assignment function, and a second-order leapfrog in ln a.

Readings (the paper gives the equations but not these details):
* mesh node j sits at x = j h (h = L/N); positions live in [0, L); axis d of
  the mesh is coordinate d of the particle arrays ``pos[d]``;
* deterministic deposit: s = x (N/L) in float64, i = floor(s) mod N,
  f = s - floor(s), per-axis weights (1-f, f), the 3D weight evaluated as
  (w_x w_y) w_z without fused multiply-add, quantised Q = rint(W 2^40)
  (round half to even) and summed as 64-bit integers;
* delta = Q * (2^-40 N^3/Np) - 1, then its sample mean is removed;
* the force mesh is g = -(c/H0)^2 grad phi (units with H0 = 1, lengths in
  Mpc/h), gradient spectral with i k_i -> 0 at the Nyquist index;
* leapfrog with momenta p = a^2 dx/dt held at half steps:
  dp/dln a = g / E(a) (kick at a_n with the full step), then
  dx/dln a = p / (a^2 E(a)) evaluated at a_{n+1/2} = a_n e^{dlna/2} (drift),
  then positions are wrapped into [0, L);
* force laws: nlDGP (Eqs. FullDGP1-2), lDGP (their linear form), GRH (Eq. GRPoisson with the DGP
  expansion history) and GR (standard gravity with its own expansion history, read as flat
  LCDM with the same Omega_m0, in the Poisson coefficient and in the time integration).
"""
import math
import numpy as np

from . import spectral as sp
from .cosmology import coefficients, hubble_E, hubble_E_lcdm, omega_m_lcdm, C_OVER_H0
from . import field as fld

QBITS = 40
FORCE_NLDGP, FORCE_LDGP, FORCE_GRH, FORCE_GR = 0, 1, 2, 3


def _cell_and_weights(pos, n, box):
    """Per-axis lower cell index and the two CIC weights (Eq. CIC tent window)."""
    scale = float(n) / float(box)
    s = np.asarray(pos, dtype=np.float64) * scale
    fl = np.floor(s)
    f = s - fl
    i0 = np.mod(fl.astype(np.int64), n)
    i1 = np.mod(i0 + 1, n)
    return (i0, i1), (1.0 - f, f)


def cic_deposit_fixed(pos, n, box):
    """Integer CIC deposit: int64 grid of sum over particles of rint(W * 2^40).

    pos: (3, Np) array (float32 or float64).  Returns int64 (n, n, n).
    """
    (i0, i1), (w0, w1) = _cell_and_weights(pos, n, box)
    idx = (i0, i1)
    wts = (w0, w1)
    grid = np.zeros(n * n * n, dtype=np.int64)
    scale = float(2 ** QBITS)
    for a in (0, 1):
        for b in (0, 1):
            wxy = wts[a][0] * wts[b][1]          # product rounded before the third factor
            for c in (0, 1):
                wgt = wxy * wts[c][2]
                q = np.rint(wgt * scale).astype(np.int64)
                flat = (idx[a][0] * n + idx[b][1]) * n + idx[c][2]
                np.add.at(grid, flat, q)
    return grid.reshape(n, n, n)


def delta_from_counts(grid, n_particles):
    """delta = Q 2^-40 N^3/Np - 1, sample mean removed (float64)."""
    n = grid.shape[0]
    qscale = math.ldexp(float(n) ** 3 / float(n_particles), -QBITS)
    d = grid.astype(np.float64) * qscale - 1.0
    return d - d.mean()


def deposit(pos, n, box):
    """Deposit particles and return (int64 grid, delta)."""
    grid = cic_deposit_fixed(pos, n, box)
    return grid, delta_from_counts(grid, np.asarray(pos).shape[1])


def phi_spectrum(delta, u, box, prm, omega_m0, a, mode=FORCE_NLDGP):
    """Fourier-space Newtonian potential phi(k) (units of c^2).

    nlDGP / lDGP: Eq. FullDGP1 with sqrt(-lapbar) -> kbar and C = -u/kbar^2:
      -(kbar^2 + kbar/eta) phi = (3/2)((eta-1)/eta) delta - u/(2 eta) + c2 u/kbar.
    lDGP uses the linear u (Sec. II, Eq. LinearDGP is its expansion).
    GRH: Eq. GRPoisson with the DGP background, -kbar^2 phi = (3/2)((eta-1)/eta) delta.
    GR: Eq. GRPoisson with its own (flat LCDM) background: kbar = c k/(a H_LCDM) and
    Omega_m(a) of LCDM, -kbar^2 phi = (3/2) Omega_m(a) delta.
    k = 0 -> 0.
    """
    n = delta.shape[-1]
    c = coefficients(omega_m0, a)
    dk = sp.fft3(fld.remove_mean(delta))
    if mode == FORCE_GR:
        kb = np.broadcast_to(sp.kbar(n, box, C_OVER_H0 / (a * hubble_E_lcdm(omega_m0, a))), dk.shape)
        num = 1.5 * omega_m_lcdm(omega_m0, a) * dk
        return np.where(kb > 0, -num / np.where(kb > 0, kb * kb, 1.0), 0.0)
    kb = np.broadcast_to(sp.kbar(n, box, c.kappa), dk.shape)
    ikb = sp.inv_kbar(n, box, c.kappa)
    om = 1.5 * (c.eta - 1.0) / c.eta
    if mode == FORCE_GRH:
        num = om * dk
        den = kb * kb
    else:
        if mode == FORCE_LDGP:
            _, sk, _ = fld.source(delta, box, prm)
            uk = sp.fft3(fld.linear_solution(sk, box, prm))
        else:
            uk = sp.fft3(u)
        c2 = c.c2 if prm.nonlocal_terms else 0.0
        inv_eta_nl = 1.0 / c.eta if prm.nonlocal_terms else 0.0
        num = om * dk - uk / (2.0 * c.eta) + c2 * uk * ikb
        den = kb * kb + kb * inv_eta_nl
    phik = np.where(kb > 0, -num / np.where(kb > 0, den, 1.0), 0.0)
    return phik


def force_mesh(phik, box):
    """g_i = -(c/H0)^2 d_i phi on the mesh (Sec. III A: grad phi = i k phi, 3 inverse FFTs)."""
    n = phik.shape[0]
    return np.stack([-(C_OVER_H0 ** 2) * sp.ifft3(sp.gradient_multiplier(i, n, box) * phik, n)
                     for i in range(3)])


def cic_interpolate(mesh, pos, box):
    """Interpolate mesh fields (m, n, n, n) to particles with the CIC weights: (m, Np)."""
    mesh = np.asarray(mesh, dtype=np.float64)
    n = mesh.shape[-1]
    (i0, i1), (w0, w1) = _cell_and_weights(pos, n, box)
    idx = (i0, i1)
    wts = (w0, w1)
    out = np.zeros((mesh.shape[0], idx[0].shape[1]))
    for a in (0, 1):
        for b in (0, 1):
            wxy = wts[a][0] * wts[b][1]
            for c in (0, 1):
                wgt = wxy * wts[c][2]
                out += wgt * mesh[:, idx[a][0], idx[b][1], idx[c][2]]
    return out


def kick_drift(pos, vel, force, a, dlna, omega_m0, box, hubble=hubble_E):
    """One leapfrog step in ln a (readings in the module docstring); ``hubble`` is the background
    E(a) of the run (the DGP one, or LCDM for standard gravity).  Returns (pos, vel)."""
    dt = pos.dtype
    e_n = hubble(omega_m0, a)
    a_half = a * math.exp(0.5 * dlna)
    e_half = hubble(omega_m0, a_half)
    kick = dlna / e_n
    drift = dlna / (a_half * a_half * e_half)
    v = np.asarray(vel, dtype=np.float64) + kick * force
    x = np.asarray(pos, dtype=np.float64) + drift * v
    x = x - box * np.floor(x / box)
    v = v.astype(dt)
    x = x.astype(dt)
    x = np.where(x >= dt.type(box), x - dt.type(box), x).astype(dt)
    return x, v


def pm_forces(delta, u, pos, box, prm, omega_m0, a, mode=FORCE_NLDGP):
    """Force on particles: modified Poisson, spectral gradient, CIC interpolation."""
    phik = phi_spectrum(delta, u, box, prm, omega_m0, a, mode)
    return cic_interpolate(force_mesh(phik, box), pos, box), phik


def step(pos, vel, u_state, a, dlna, box, n, prm, omega_m0, mode=FORCE_NLDGP):
    """One PM step: deposit -> field solve (warm start when u_state is given) ->
    forces -> interpolation -> kick-drift.  Returns (pos, vel, u, info)."""
    _, delta = deposit(pos, n, box)
    if mode == FORCE_NLDGP:
        p = prm if u_state is None else prm.with_(init=fld.INIT_WARM)
        u, info = fld.solve(delta, box, p, u0=u_state)
    else:
        u, info = u_state, None
    force, _ = pm_forces(delta, u, pos, box, prm, omega_m0, a, mode)
    x, v = kick_drift(pos, vel, force, a, dlna, omega_m0, box, hubble_E_lcdm if mode == FORCE_GR else hubble_E)
    return x, v, u, info


def run(pos, vel, a_start, dlna, n_steps, a_switch, box, n, omega_m0, lam, tol, max_iter=100, w=1.0 / 3.0,
        spherical=False, mode=FORCE_NLDGP):
    """n_steps PM steps from a_start (Sec. III A time stepping; Sec. III D: the linearised DGP
    Poisson equation at early times, the full nonlinear solve from a_switch on).  Step k runs at
    a_k = a_start exp(k dlna) with the coefficients of a_k; each nonlinear solve after the first
    starts from the previous step's field.  spherical: the spherical approximation (Eq. SphPoi)
    replaces the full solve.  mode other than nlDGP: every step uses that force law (the lDGP,
    GRH and GR comparison runs; no switch).  Returns (pos, vel, u, [SolveInfo or None per step])."""
    u = None
    infos = []
    for k in range(n_steps):
        a = a_start * math.exp(k * dlna)
        prm = fld.SolveParams.from_cosmology(omega_m0, a, lam=lam, w=w, tol=tol, max_iter=max_iter)
        if mode != FORCE_NLDGP:
            pos, vel, _, _ = step(pos, vel, None, a, dlna, box, n, prm, omega_m0, mode=mode)
            infos.append(None)
        elif a < a_switch:
            pos, vel, _, _ = step(pos, vel, None, a, dlna, box, n, prm, omega_m0, mode=FORCE_LDGP)
            infos.append(None)
        elif spherical:
            _, delta = deposit(pos, n, box)
            u = fld.spherical_first_update(delta, box, prm)
            force, _ = pm_forces(delta, u, pos, box, prm, omega_m0, a, FORCE_NLDGP)
            pos, vel = kick_drift(pos, vel, force, a, dlna, omega_m0, box)
            infos.append(None)
        else:
            pos, vel, u, info = step(pos, vel, u, a, dlna, box, n, prm, omega_m0)
            infos.append(info)
    return pos, vel, u, infos
