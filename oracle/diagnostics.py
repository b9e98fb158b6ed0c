"""Diagnostics of a solved brane-bending field (CPU oracle, float64; test infrastructure only).

* Ellipticity (Appendix, Eq. EllipticMatrix): Eq. FullDGP2 with the nonlinear coefficient
  lam is F = lam[(lap C)^2 - (h_ij)^2] + alpha lap C + ... ; the matrix of dF/d(h_ij) is
  (2 lam u + alpha) I - 2 lam h, u = lap C.  The equation is elliptic at a point when its three
  eigenvalues share one sign; the fraction of points where they do not is reported.
* c of Eq. cdef, c = alpha eta / (3 (eta - 1)) u, and the ratio P_c / P_m of its power spectrum
  to that of delta (Sec. IV, the Vainshtein suppression plot).
* Delta_gradC of Eq. DGradC: 4 pi k^5 P_C(k) at the bin centres of the binned estimator.
"""
import numpy as np

from . import field as fld
from . import power
from .cosmology import coefficients


def ellipticity_matrix(u, box, prm):
    """(..., 3, 3) array of dF/d(h_ij) at every point."""
    h, _ = fld.hessian_fields(u, box, prm)
    mat = np.empty(u.shape + (3, 3))
    for (i, j) in fld.PAIRS:
        mat[..., i, j] = -2.0 * prm.lam * h[i, j]
        mat[..., j, i] = -2.0 * prm.lam * h[i, j]
    for i in range(3):
        mat[..., i, i] += 2.0 * prm.lam * u + prm.alpha
    return mat


def nonelliptic_fraction(u, box, prm):
    """Fraction of points whose ellipticity matrix has eigenvalues of mixed sign (or zero),
    and the smallest |eigenvalue| at each point (to flag decisions near the boundary)."""
    ev = np.linalg.eigvalsh(ellipticity_matrix(u, box, prm).reshape(-1, 3, 3))
    elliptic = np.all(ev > 0, axis=1) | np.all(ev < 0, axis=1)
    return 1.0 - np.count_nonzero(elliptic) / float(ev.shape[0]), np.min(np.abs(ev), axis=1)


def c_field_coefficient(omega_m0, a):
    """alpha eta / (3 (eta - 1)) of Eq. cdef."""
    c = coefficients(omega_m0, a)
    return c.alpha * c.eta / (3.0 * (c.eta - 1.0))


def pc_over_pm(delta, u, box, omega_m0, a, nbins=64):
    """P_c(k) / P_m(k) per bin (0 where P_m is 0)."""
    coef = c_field_coefficient(omega_m0, a)
    pc, _, _ = power.power_spectrum(coef * u, box, nbins)
    pm, _, _ = power.power_spectrum(delta, box, nbins)
    return np.where(pm > 0, pc / np.where(pm > 0, pm, 1.0), 0.0)


def delta_gradc(u, box, prm, nbins=64):
    """4 pi k_b^5 P_C(k_b) with C = lap^{-1} u (the binned estimator's k centres)."""
    pk, _, kc = power.power_spectrum(fld.c_from_u(u, box, prm), box, nbins)
    return 4.0 * np.pi * kc ** 5 * pk
