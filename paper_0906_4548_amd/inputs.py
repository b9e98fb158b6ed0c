"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers and shapes them into density fields and
particle loads with the statistics of the paper's workloads; it contains none
of the field-solve or PM arithmetic.  Everything is float64 NumPy on the host;
callers copy the arrays to the device themselves.

* ``gaussian_field``: Gaussian random field with a power-law (optionally
  cut-off) spectrum, colouring seeded white noise in Fourier space, k = 0 -> 0.
* ``lognormal_delta``: delta = exp(g - sigma^2/2) - 1 of a Gaussian g with
  P(k) ~ k^slope normalised to sample rms exactly sigma (the log-normal stand-in
  for a nonlinear density field with deep voids, delta > -1).
* ``zeldovich_load``: particles on a lattice q = (i + 1/2) L / n, displaced by
  Psi with Psi(k) = i k delta_L(k) / k^2 (Nyquist of the odd factor -> 0),
  delta_L Gaussian with P ~ k^slope exp(-k^2/k_c^2), rescaled so that the rms of
  |Psi| over particles equals ``rms_disp``.  Returns the wrapped positions and
  Psi (velocities are Psi times a growth factor the caller chooses).
"""
import numpy as np


def _kmag(n, box):
    kf = 2.0 * np.pi / box
    full = kf * np.fft.fftfreq(n, 1.0 / n)
    half = kf * np.arange(n // 2 + 1)
    return full[:, None, None], full[None, :, None], half[None, None, :]


def gaussian_field(n, box, seed, slope=-2.0, kc=None):
    """Real Gaussian field on an n^3 mesh with P(k) ~ k^slope [exp(-k^2/kc^2)]."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    kx, ky, kz = _kmag(n, box)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    safe = np.where(k > 0, k, 1.0)
    amp = np.where(k > 0, safe ** (0.5 * slope), 0.0)
    if kc is not None:
        amp = amp * np.exp(-0.5 * (k / kc) ** 2)
    return np.fft.irfftn(np.fft.rfftn(white) * amp, s=(n, n, n), axes=(0, 1, 2))


def lognormal_delta(n, box, sigma, seed, slope=-2.0):
    """Log-normal density contrast; the Gaussian has sample rms exactly ``sigma``."""
    g = gaussian_field(n, box, seed, slope)
    g *= sigma / np.sqrt(np.mean(g * g))
    return np.exp(g - 0.5 * sigma * sigma) - 1.0


def zeldovich_load(n_side, box, seed, slope=-1.5, kc=1.0, rms_disp=2.0, dtype=np.float64, block=0):
    """Zel'dovich particle load: (positions (3, Np) of ``dtype``, displacement (3, Np) float64).

    Particles are stored in lattice order (axis 2 fastest); with ``block`` = b > 0 they are
    stored in Lagrangian blocks of b^3 lattice sites instead (blocks in lattice order, sites
    in lattice order inside a block), a spatially coherent order.
    """
    n = n_side
    dl = gaussian_field(n, box, seed, slope, kc)
    dk = np.fft.rfftn(dl)
    kx, ky, kz = _kmag(n, box)
    k2 = kx * kx + ky * ky + kz * kz
    safe = np.where(k2 > 0, k2, 1.0)
    kf = 2.0 * np.pi / box
    nyq = 0.5 * n * kf
    psi = []
    for kd in (kx, ky, kz):
        odd = np.where(np.abs(np.abs(kd) - nyq) < 1e-9 * kf, 0.0, kd)
        mult = np.where(k2 > 0, 1j * odd / safe, 0.0)
        psi.append(np.fft.irfftn(dk * mult, s=(n, n, n), axes=(0, 1, 2)))
    psi = np.stack(psi).reshape(3, -1)
    psi *= rms_disp / np.sqrt(np.mean(np.sum(psi * psi, axis=0)))
    q1 = (np.arange(n) + 0.5) * (box / n)
    qx, qy, qz = np.meshgrid(q1, q1, q1, indexing='ij')
    q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()])
    x = q + psi
    x = x - box * np.floor(x / box)
    x = x.astype(dtype)
    x = np.where(x >= dtype(box), x - dtype(box), x).astype(dtype)
    if block:
        if n % block:
            raise ValueError("block must divide n_side")
        m = n // block
        order = np.arange(n ** 3).reshape(m, block, m, block, m, block).transpose(0, 2, 4, 1, 3, 5).ravel()
        x, psi = x[:, order], psi[:, order]
    return np.ascontiguousarray(x), np.ascontiguousarray(psi)


def random_cells(n, count, seed):
    """``count`` distinct flat cell indices of an n^3 mesh."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n * n * n, size=count, replace=False))
