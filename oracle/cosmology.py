"""Background expansion and field-equation coefficients (oracle; test infrastructure).

Follows Sec. II "Equations of Motion": the self-accelerating DGP Friedmann
equation (Eq. DGPFriedmann) with r_c H0 = 1/(1 - Omega_m0), and the definitions
of eta, beta, alpha, the nonlocal coefficients of Eqs. FullDGP1 / FullDGP2, the
acceleration parameter q and the effective Newton constant (Eq. Geff).

Units: H0 = 1 for time; lengths in Mpc/h; c/H0 = 2997.92458 Mpc/h.  The barred
gradient of the paper is grad/(aH) with c = 1, so a comoving wavenumber k
[h/Mpc] maps to kbar = kappa * k with kappa = (c/H0) / (a E(a)).
"""
import math
from dataclasses import dataclass, asdict

C_OVER_H0 = 2997.92458  # Mpc/h


def hubble_E(omega_m0, a):
    """E(a) = H/H0 solving Eq. DGPFriedmann, H^2 = H/r_c + (8 pi G/3) rho_m.

    In units of H0 with r_c H0 = 1/(1-Om0):  E^2 = (1-Om0) E + Om0 a^-3,
    whose positive root is [(1-Om0) + sqrt((1-Om0)^2 + 4 Om0 a^-3)] / 2.
    """
    om = float(omega_m0)
    b = 1.0 - om
    return 0.5 * (b + math.sqrt(b * b + 4.0 * om / a ** 3))


def hubble_E_lcdm(omega_m0, a):
    """E(a) of the standard-gravity comparison runs (GR with its own expansion history): flat
    LCDM with the same Omega_m0 (Sec. III A parameters), E^2 = Om0 a^-3 + (1 - Om0)."""
    om = float(omega_m0)
    return math.sqrt(om / a ** 3 + (1.0 - om))


def omega_m_lcdm(omega_m0, a):
    """Omega_m(a) = Om0 a^-3 / E^2 of the flat LCDM background."""
    return float(omega_m0) / a ** 3 / hubble_E_lcdm(omega_m0, a) ** 2


def eta_of(omega_m0, a):
    """eta = r_c H (Sec. II) = E(a) / (1 - Om0)."""
    return hubble_E(omega_m0, a) / (1.0 - omega_m0)


@dataclass
class Coefficients:
    """Scalar coefficients of Eqs. FullDGP1 / FullDGP2 (Sec. II)."""
    omega_m0: float
    a: float
    E: float       # H/H0
    eta: float     # r_c H
    beta: float    # (2 eta^2 - 2 eta - 1) / (eta (2 eta - 1))
    alpha: float   # 3 (2 eta^2 - 2 eta + 1) / (eta (2 eta - 1))
    A: float       # 3 (eta - 1) / eta : source coefficient of Eq. FullDGP2
    gamma: float   # 3 beta (eta - 1) / (2 eta - 1) : coefficient of sqrt(-lap) C in Eq. FullDGP2
    c2: float      # (3 eta^2 - 5 eta + 1) / (2 eta^2 (2 eta - 1)) : coefficient of sqrt(-lap) C in Eq. FullDGP1
    q: float       # acceleration parameter (2 - eta) / (2 eta - 1)
    kappa: float   # c / (a H) in Mpc/h

    def as_dict(self):
        return asdict(self)


def coefficients(omega_m0, a):
    """All coefficients at scale factor a (Sec. II definitions)."""
    E = hubble_E(omega_m0, a)
    eta = E / (1.0 - omega_m0)
    den = eta * (2.0 * eta - 1.0)
    beta = (2.0 * eta * eta - 2.0 * eta - 1.0) / den
    alpha = 3.0 * (2.0 * eta * eta - 2.0 * eta + 1.0) / den
    A = 3.0 * (eta - 1.0) / eta
    gamma = 3.0 * beta * (eta - 1.0) / (2.0 * eta - 1.0)
    c2 = (3.0 * eta * eta - 5.0 * eta + 1.0) / (2.0 * eta * eta * (2.0 * eta - 1.0))
    q = (2.0 - eta) / (2.0 * eta - 1.0)
    kappa = C_OVER_H0 / (a * E)
    return Coefficients(omega_m0, a, E, eta, beta, alpha, A, gamma, c2, q, kappa)


def omega_m_of_a(omega_m0, a):
    """Omega_m(a) = (eta - 1)/eta, from dividing Eq. DGPFriedmann by H^2."""
    eta = eta_of(omega_m0, a)
    return (eta - 1.0) / eta


def w_zero_discriminant(omega_m0, a):
    """Eq. ZeroDis: the split w that zeroes the C-free part of Eq. NewDis at delta = -1."""
    c = coefficients(omega_m0, a)
    return 1.0 - c.alpha ** 2 * c.eta / (12.0 * (c.eta - 1.0))


def discriminant_c_free(omega_m0, a, w, delta=-1.0):
    """C-independent part of the discriminant of Eq. NewDis (nonlocal terms dropped):
    alpha^2 + 4 (1 - w) * 3 (eta - 1)/eta * delta.  w = 0 is Eq. Discweq0 (Fig. 2)."""
    c = coefficients(omega_m0, a)
    return c.alpha ** 2 + 4.0 * (1.0 - w) * c.A * delta


def monge_ampere_det_2d(omega_m0, a, delta=-1.0):
    """Eq. Det2D: determinant of the 2D ellipticity matrix, alpha^2 + 6 (eta-1)/eta delta."""
    c = coefficients(omega_m0, a)
    return c.alpha ** 2 + 6.0 * (c.eta - 1.0) / c.eta * delta


def geff_ratio(omega_m0, a, k):
    """G_eff / G of Eq. Geff at comoving wavenumber k [h/Mpc], written with r_c as printed:
    the scale-dependent term carries 3 a / (k r_c), r_c = (c/H0) / (1 - Omega_m0)."""
    c = coefficients(omega_m0, a)
    r_c = C_OVER_H0 / (1.0 - omega_m0)
    first = (2.0 * c.eta * (2.0 + c.q) - 3.0) / (2.0 * c.eta * (2.0 + c.q) - 4.0)
    second = (3.0 * a / (k * r_c)) * ((c.eta * (1.0 + c.q) - 1.0) / (c.eta * (2.0 + c.q) - 2.0)) ** 2
    return 1.0 / (first + second)
