"""Plain CPU FP64 oracle for the DGP FFT-relaxation field solve and the PM step.

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.  The
product path (the HIP library and its Python binding) never imports, links or
calls anything here, and nothing here imports the product path.

Everything is written for a reader holding the paper (Chan & Scoccimarro,
"Large-Scale Structure in Brane-Induced Gravity II. Numerical Simulations"):
each function cites the section / equation it follows.  Arithmetic is float64
NumPy; FFTs are numpy.fft (pocketfft).  No blocking, fusion or reordering beyond
what the paper's equations state.

Modules
-------
cosmology  background and the coefficients of the field equations (Sec. II)
spectral   wavenumber grids, the spectral multipliers and a brute-force DFT
field      the FFT-relaxation solve (Sec. III B, III C) and its pieces
newton     an independent Newton-Krylov / dense-Newton solver of the same
           discrete equation (a cross-check of the relaxation's fixed point)
pm         CIC deposit / interpolation, modified Poisson, forces, leapfrog (Sec. III A)
power      binned power spectrum (Sec. IV)
adjoint    Jacobian, dense implicit adjoint and CIC adjoints
"""

from . import cosmology, spectral, field, newton, pm, power, adjoint  # noqa: F401
