"""Binned power spectrum (oracle; test infrastructure).

The paper measures P(k) of the density and of the normalised brane-bending
mode (power-spectrum section, Eq. cdef) but does not state its estimator.
Reading used here (and by the GPU path):
* nbins logarithmic bins between the fundamental k_f = 2 pi / L and the mesh
  Nyquist k_f N/2, edges k_f (N/2)^(b/nbins), b = 0..nbins;
* a mode with integer mode vector m (|m_d| <= N/2) belongs to bin b when
  T_b <= |m|^2 < T_{b+1}, with integer thresholds T_b = ceil((N/2)^(2b/nbins));
  the last bin also holds |m|^2 = (N/2)^2; k = 0 and |m| > N/2 are excluded;
  (a lower-inclusive bin in |k| is exactly this test on the integer |m|^2);
* modes are counted over the full spectrum (each rfft mode with 0 < m_2 < N/2
  stands for itself and its conjugate);
* P_b = (L^3 / N^6) * mean over the bin's modes of |F(k)|^2; no shot-noise or
  window correction.  Empty bins give P_b = 0 with count 0.
"""
import math
import numpy as np

from . import spectral as sp


def bin_thresholds(n, nbins=64):
    """Integer thresholds T_b on |m|^2, b = 0..nbins (T_nbins is (N/2)^2 + 1)."""
    half = n // 2
    t = [int(math.ceil(float(half) ** (2.0 * b / nbins))) for b in range(nbins + 1)]
    t[nbins] = half * half + 1
    return np.array(t, dtype=np.int64)


def mode_bins(n, nbins=64):
    """Bin index of every rfft mode (-1 for excluded modes) and its multiplicity."""
    m0, m1, m2 = sp.mode_numbers(n)
    msq = (m0 * m0 + m1 * m1 + m2 * m2).astype(np.int64)
    msq = np.broadcast_to(msq, (n, n, n // 2 + 1))
    t = bin_thresholds(n, nbins)
    b = np.searchsorted(t, msq, side='right') - 1
    b = np.where((msq >= t[0]) & (msq < t[-1]), b, -1)
    mult = np.where((m2 == 0) | (m2 == n // 2), 1, 2) * np.ones_like(msq)
    return b, mult


def power_spectrum(field, box, nbins=64):
    """(P_b, counts_b, k-centre of each bin) of a real mesh field."""
    n = field.shape[-1]
    fk = sp.fft3(field)
    b, mult = mode_bins(n, nbins)
    p2 = (fk.real ** 2 + fk.imag ** 2) * mult
    sel = b >= 0
    sums = np.bincount(b[sel], weights=p2[sel], minlength=nbins)
    cnt = np.bincount(b[sel], weights=mult[sel], minlength=nbins)
    pk = np.where(cnt > 0, sums / np.where(cnt > 0, cnt, 1.0), 0.0) * box ** 3 / float(n) ** 6
    kf = 2.0 * np.pi / box
    edges = kf * (n / 2.0) ** (np.arange(nbins + 1) / nbins)
    return pk, cnt.astype(np.int64), np.sqrt(edges[:-1] * edges[1:])


def power_spectrum_grad(field, grad_pk, box, nbins=64):
    """d(sum_b grad_pk[b] P_b)/d field for a real mesh field.

    P_b = c_b sum_{full k in b} |F(k)|^2 with c_b = L^3/(N^6 count_b); the
    gradient of sum_k |F(k)|^2 over a set closed under k -> -k is
    2 N^3 F^{-1}[1_set F field].
    """
    n = field.shape[-1]
    _, cnt, _ = power_spectrum(field, box, nbins)
    b, _ = mode_bins(n, nbins)
    coef = np.where(cnt > 0, np.asarray(grad_pk, dtype=np.float64) * box ** 3
                    / (float(n) ** 6 * np.where(cnt > 0, cnt, 1)), 0.0)
    mult = np.where(b >= 0, coef[np.maximum(b, 0)], 0.0) * 2.0 * float(n) ** 3
    return sp.ifft3(mult * sp.fft3(field), n)
