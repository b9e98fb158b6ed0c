"""Wavenumber grids and spectral multipliers on the periodic mesh (oracle; test infrastructure).

The paper evaluates the Hessian of C, the nonlocal operators sqrt(-lap) and
lap^{-1/2}, and the force gradient as multipliers in Fourier space:
  grad_i grad_j C (k) = -k_i k_j C(k)          (Sec. III B, the Hessian equation)
  sqrt(-lap) -> kbar,  lap^{-1/2} -> 1/kbar     (Sec. II, after the definition of grad-bar)
  grad phi -> i k phi                           (Sec. III A)
It uses "the same symbol" for a field and its transform.

Conventions (readings of what the paper leaves open):
* forward transform unnormalised, inverse carries 1/N^3 (numpy.fft);
* the k = 0 multiplier of k_i k_j / k^2, 1/kbar and 1/kbar^2 is 0;
* at a Nyquist index (|n| = N/2) every multiplier that is odd in that
  component is 0: the mixed Hessian terms (i != j) and the gradient i k_i.
  This keeps every spectrum Hermitian, so each inverse transform is real.

Transforms are numpy's rfftn / irfftn over all three axes (last axis halved).  ``fft_workers``
switches the same transforms to scipy.fft with a number of threads (used only to time the oracle
on all host cores; results agree to rounding).
"""
import contextlib

import numpy as np

_WORKERS = None


@contextlib.contextmanager
def fft_workers(workers):
    """Within the block, fft3 / ifft3 run as scipy.fft transforms on `workers` threads."""
    global _WORKERS
    old, _WORKERS = _WORKERS, workers
    try:
        yield
    finally:
        _WORKERS = old


def fft3(x):
    """Forward 3D real-to-complex transform (unnormalised)."""
    if _WORKERS:
        import scipy.fft
        return scipy.fft.rfftn(np.asarray(x, dtype=np.float64), axes=(-3, -2, -1), workers=_WORKERS)
    return np.fft.rfftn(np.asarray(x, dtype=np.float64), axes=(-3, -2, -1))


def ifft3(xk, n):
    """Inverse 3D complex-to-real transform (carries 1/N^3)."""
    if _WORKERS:
        import scipy.fft
        return scipy.fft.irfftn(xk, s=(n, n, n), axes=(-3, -2, -1), workers=_WORKERS)
    return np.fft.irfftn(xk, s=(n, n, n), axes=(-3, -2, -1))


def mode_numbers(n):
    """Integer mode numbers along the three axes of the rfft grid, broadcastable.

    Axes 0 and 1: 0..N/2-1, -N/2..-1 (the Nyquist index is -N/2).  Axis 2: 0..N/2.
    """
    full = np.fft.fftfreq(n, 1.0 / n).round().astype(np.int64)
    half = np.arange(n // 2 + 1, dtype=np.int64)
    return (full[:, None, None], full[None, :, None], half[None, None, :])


def wavevectors(n, box):
    """Comoving wave-vector components k_d = 2 pi n_d / L [h/Mpc], broadcastable."""
    kf = 2.0 * np.pi / box
    return tuple(kf * m.astype(np.float64) for m in mode_numbers(n))


def k_squared(n, box):
    kx, ky, kz = wavevectors(n, box)
    return kx * kx + ky * ky + kz * kz


def is_nyquist(n):
    """Boolean masks (broadcastable) of the Nyquist index along each axis."""
    return tuple(np.abs(m) == n // 2 for m in mode_numbers(n))


def hessian_multiplier(i, j, n, box):
    """Multiplier m_ij = k_i k_j / k^2 taking u = lap C to grad_i grad_j C.

    From grad_ij C(k) = -k_i k_j C(k) and u(k) = -k^2 C(k) (Sec. III B); the
    factor kappa of the barred gradient cancels.  k = 0 -> 0; mixed terms at a
    Nyquist index of i or j -> 0.
    """
    k = wavevectors(n, box)
    k2 = k_squared(n, box)
    safe = np.where(k2 > 0, k2, 1.0)
    m = np.where(k2 > 0, k[i] * k[j] / safe, 0.0)
    if i != j:
        nyq = is_nyquist(n)
        m = np.where(nyq[i] | nyq[j], 0.0, m)
    return np.broadcast_to(m, (n, n, n // 2 + 1)).copy()


def kbar(n, box, kappa):
    """kbar = kappa |k| (the eigenvalue of sqrt(-lapbar))."""
    return kappa * np.sqrt(k_squared(n, box)) * np.ones((1, 1, 1))


def inv_kbar(n, box, kappa):
    """1/kbar with the k = 0 mode set to 0."""
    kb = np.broadcast_to(kbar(n, box, kappa), (n, n, n // 2 + 1))
    return np.where(kb > 0, 1.0 / np.where(kb > 0, kb, 1.0), 0.0)


def gradient_multiplier(i, n, box):
    """i k_i of the spectral gradient (Sec. III A), 0 at the Nyquist index of axis i."""
    k = wavevectors(n, box)
    nyq = is_nyquist(n)
    m = np.where(nyq[i], 0.0, k[i])
    return np.broadcast_to(1j * m, (n, n, n // 2 + 1)).copy()


def dft3_bruteforce(x):
    """Direct O(N^6) 3D DFT, X(k) = sum_x x e^{-2 pi i k.x/N}, for pinning the FFT.

    Returns the full (N, N, N) complex spectrum.  Only for tiny N.
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    idx = np.arange(n)
    w = np.exp(-2j * np.pi * np.outer(idx, idx) / n)  # 1D DFT matrix, built from its definition
    out = np.zeros((n, n, n), dtype=np.complex128)
    for k0 in range(n):
        for k1 in range(n):
            for k2 in range(n):
                ph = w[k0][:, None, None] * w[k1][None, :, None] * w[k2][None, None, :]
                out[k0, k1, k2] = np.sum(x * ph)
    return out
