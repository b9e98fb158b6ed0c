"""FFT-relaxation solve of the brane-bending equation (oracle; test infrastructure).

Follows Sec. III B "FFT-Relaxation Method" and Sec. III C "Splitting the
Nonlinear Terms" of the paper, step by step, in plain float64 NumPy.

The unknown is u = lapbar C (the paper's nabla-bar^2 C).  Eq. FullDGP2, with a
coefficient lam in front of its two quadratic terms (lam = 1 is the paper), reads

    lam [u^2 - sum_ij h_ij^2] + alpha u + gamma Nf = S                       (*)

with h_ij = gradbar_i gradbar_j C (spectral Hessian of u), Nf = sqrt(-lapbar) C
(the nonlocal term, -u(k)/kbar in Fourier space), gamma = 3 beta (eta-1)/(2eta-1)
and S = A (1 - beta lapbar^{-1/2}) delta, A = 3 (eta-1)/eta.

Readings of points the paper leaves open (each is applied identically by the
GPU path):
* residual norm: r = <|R|> / eps with eps of Eq. normres (the plain average <R>
  vanishes identically on a periodic mesh, so the absolute value is taken, as
  in eps itself); for eps = 0 (uniform delta) r is 0 when R = 0, else +inf;
* R uses the full pointwise iterate u (no re-projection of its mean);
* delta's sample mean is removed first; k = 0 multipliers are 0;
* the root of Eq. nabla^2Cwpara is evaluated in the algebraically identical
  form 2 B' / (alpha + sqrt(Delta)), which has no cancellation when
  4 (1-w) lam B' << alpha^2;
* a bad point (Delta < 0) takes Delta = 0, i.e. the parabola vertex
  u = -alpha / (2 (1-w) lam) (Sec. III C "set the discriminant to zero");
* damping omega (u <- (1-omega) u + omega u_new) is 1 in the paper;
* stop when r <= tol; when bad points have occurred and the residual stops
  decreasing, stop and return the minimum-residual iterate (Sec. III C, Fig. 4
  discussion); at max_iter return the minimum-residual iterate.
"""
from dataclasses import dataclass, field as dc_field, replace
import numpy as np

from . import spectral as sp
from .cosmology import coefficients

INIT_LINEAR, INIT_ZERO, INIT_WARM = 0, 1, 2
STATUS_OK, STATUS_NOT_CONVERGED, STATUS_BAD_POINTS = 0, 1, 2


@dataclass
class SolveParams:
    """Inputs of one field solve; the coefficient fields follow Sec. II."""
    alpha: float
    beta: float
    A: float
    gamma: float
    kappa: float
    lam: float = 1.0          # coefficient of the quadratic terms (1 = paper)
    w: float = 1.0 / 3.0      # split parameter, Eq. FullDGP2wpara (1/3 = paper's choice)
    omega: float = 1.0        # damping (paper: none)
    tol: float = 1e-2         # normalised-residual target (paper: 1 %)
    max_iter: int = 100
    init: int = INIT_LINEAR
    nonlocal_terms: bool = True   # keep the sqrt(-lap) / lap^{-1/2} terms

    @staticmethod
    def from_cosmology(omega_m0, a, **kw):
        c = coefficients(omega_m0, a)
        return SolveParams(alpha=c.alpha, beta=c.beta, A=c.A, gamma=c.gamma, kappa=c.kappa, **kw)

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def gamma_eff(self):
        return self.gamma if self.nonlocal_terms else 0.0

    @property
    def beta_eff(self):
        return self.beta if self.nonlocal_terms else 0.0


@dataclass
class SolveInfo:
    iters: int = 0                     # number of updates applied
    status: int = STATUS_OK
    eps: float = 0.0
    resid: float = 0.0                 # r of the returned iterate
    resid_min: float = np.inf
    bad_fraction: float = 0.0          # bad fraction of the last update computed
    mean_u: float = 0.0
    history: list = dc_field(default_factory=list)      # r_n for n = 0..
    bad_history: list = dc_field(default_factory=list)  # bad fraction of update n


def remove_mean(delta):
    """delta - <delta> (solvability on the periodic mesh)."""
    d = np.asarray(delta, dtype=np.float64)
    return d - d.mean()


def source(delta, box, prm):
    """S = A (1 - beta lapbar^{-1/2}) delta of Eq. FullDGP2, and eps of Eq. normres.

    Returns (S real-space, S spectrum, eps = <|S|>).  k = 0 -> 0.
    """
    n = delta.shape[-1]
    dk = sp.fft3(remove_mean(delta))
    mult = prm.A * (1.0 - prm.beta_eff * sp.inv_kbar(n, box, prm.kappa))
    mult[0, 0, 0] = 0.0
    sk = mult * dk
    s = sp.ifft3(sk, n)
    return s, sk, float(np.mean(np.abs(s)))


def linear_solution(sk, box, prm):
    """u of the linearised Eq. FullDGP2 (Sec. III B): (alpha - gamma/kbar) u(k) = S(k).

    From -alpha kbar^2 C + gamma kbar C = S(k) with u = -kbar^2 C.  k = 0 -> 0.
    """
    n = sk.shape[0]
    ik = sp.inv_kbar(n, box, prm.kappa)
    den = prm.alpha - prm.gamma_eff * ik
    uk = np.where(ik > 0, sk / den, 0.0)
    return sp.ifft3(uk, n)


PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def hessian_fields(u, box, prm):
    """h_ij = gradbar_i gradbar_j C for the 6 independent pairs, and Nf = sqrt(-lapbar) C.

    h_ij(k) = (k_i k_j / k^2) u(k) (Sec. III B: grad_ij C(k) = -k_i k_j C(k),
    u(k) = -kbar^2 C(k)); Nf(k) = kbar C(k) = -u(k)/kbar.  Six inverse
    transforms for the Hessian, one for Nf (Sec. III D).
    """
    n = u.shape[-1]
    uk = sp.fft3(u)
    h = {p: sp.ifft3(sp.hessian_multiplier(p[0], p[1], n, box) * uk, n) for p in PAIRS}
    nf = sp.ifft3(-sp.inv_kbar(n, box, prm.kappa) * uk, n)
    if not prm.nonlocal_terms:
        nf = np.zeros_like(nf)
    return h, nf


def hessian_square_sum(h):
    """(gradbar_ij C)^2 = sum over all i, j of h_ij^2 (off-diagonal pairs counted twice)."""
    return (h[0, 0] ** 2 + h[1, 1] ** 2 + h[2, 2] ** 2
            + 2.0 * (h[0, 1] ** 2 + h[0, 2] ** 2 + h[1, 2] ** 2))


def residual_field(u, h, nf, s, prm):
    """R = LHS - RHS of Eq. FullDGP2 (Sec. III B), quadratic terms scaled by lam."""
    return prm.lam * (u * u - hessian_square_sum(h)) + prm.alpha * u + prm.gamma_eff * nf - s


def normalized_residual(r_field, eps):
    """<|R|> / eps (Eq. normres with the absolute-value reading).

    eps = 0 only for a uniform delta (S = 0), whose exact solution is u = 0; the ratio is then
    read as 0 when R vanishes identically and +inf otherwise (the paper does not define it)."""
    num = float(np.mean(np.abs(r_field)))
    if eps == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / eps


def picard_update(u, h, nf, s, prm):
    """One FFT-relaxation update, Eqs. nabla^2Cwpara and Bwpara.

    B' = lam [sum h^2 - w u^2] - gamma Nf + S;  Delta = alpha^2 + 4 (1-w) lam B';
    u_new = (-alpha + sqrt(Delta)) / (2 (1-w) lam) (the + root, which reduces to
    linear theory), evaluated as 2 B' / (alpha + sqrt(Delta)).  Delta < 0 (a bad
    point) is set to 0.  Returns (u_new, number of bad points).
    """
    w, lam, alpha = prm.w, prm.lam, prm.alpha
    bp = lam * (hessian_square_sum(h) - w * u * u) - prm.gamma_eff * nf + s
    disc = alpha * alpha + 4.0 * (1.0 - w) * lam * bp
    bad = disc < 0.0
    root = 2.0 * bp / (alpha + np.sqrt(np.where(bad, 0.0, disc)))
    u_new = np.where(bad, -alpha / (2.0 * (1.0 - w) * lam), root)
    if prm.omega != 1.0:
        u_new = (1.0 - prm.omega) * u + prm.omega * u_new
    return u_new, int(bad.sum())


def solve(delta, box, prm, u0=None, fixed_iters=None):
    """The FFT-relaxation iteration (Eq. FFTrelax with the w-split of Sec. III C).

    Iterate n evaluates R(u^(n)); if r_n <= tol it is returned, otherwise the
    update gives u^(n+1).  ``fixed_iters`` forces exactly that many updates
    (tolerance ignored), for same-sequence comparisons.
    Returns (u, SolveInfo).
    """
    delta = np.asarray(delta, dtype=np.float64)
    n = delta.shape[-1]
    s, sk, eps = source(delta, box, prm)
    if prm.init == INIT_WARM:
        u = np.array(u0, dtype=np.float64, copy=True)
    elif prm.init == INIT_ZERO:
        u = np.zeros((n, n, n))
    else:
        u = linear_solution(sk, box, prm)
    info = SolveInfo(eps=eps)
    best_u, best_r = u, np.inf
    bad_seen = False
    max_it = prm.max_iter if fixed_iters is None else fixed_iters
    it = 0
    while True:
        h, nf = hessian_fields(u, box, prm)
        r = normalized_residual(residual_field(u, h, nf, s, prm), eps)
        info.history.append(r)
        if fixed_iters is None:
            if r <= prm.tol:
                best_u, best_r, info.status = u, r, STATUS_OK
                break
            if r < best_r:
                best_u, best_r = u, r
            elif bad_seen:
                info.status = STATUS_BAD_POINTS
                break
        else:
            best_u, best_r = u, r
        if it >= max_it:
            info.status = STATUS_NOT_CONVERGED if fixed_iters is None else STATUS_OK
            break
        u, nbad = picard_update(u, h, nf, s, prm)
        info.bad_history.append(nbad / u.size)
        info.bad_fraction = nbad / u.size
        bad_seen = bad_seen or nbad > 0
        it += 1
    info.iters = it
    info.resid = best_r
    info.resid_min = min(info.history)
    info.mean_u = float(best_u.mean())
    return best_u, info


def c_from_u(u, box, prm):
    """C = lapbar^{-1} u, i.e. C(k) = -u(k)/kbar^2 (k = 0 -> 0)."""
    n = u.shape[-1]
    ik = sp.inv_kbar(n, box, prm.kappa)
    return sp.ifft3(-ik * ik * sp.fft3(u), n)


def spherical_first_update(delta, box, prm):
    """One w = 1/3 update from u = 0 (spherical approximation, Eqs. FullDGP2sph and SphPoi).

    With u = 0 all Hessian and nonlocal terms vanish, so B' = S and
    u_1 = 2 S / (alpha + sqrt(alpha^2 + (8/3) lam S)).
    """
    p = prm.with_(w=1.0 / 3.0, omega=1.0)
    s, _, _ = source(delta, box, p)
    zero = np.zeros_like(s)
    h = {q: zero for q in PAIRS}
    u1, _ = picard_update(zero, h, zero, s, p)
    return u1
