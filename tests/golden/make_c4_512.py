"""Writes tests/golden/c4_512_fixed2.json: the oracle at the full 512^3 size, sampled.

Workload: the 512^3 Zel'dovich load of float32 particles (seed 4, box 1024 Mpc/h, one particle
per cell; the large-mesh configuration), Omega_m0 = 0.27, z = 1 (a = 0.5), w = 1/3, nonlinear
ratio r_nl = lam max|u_lin| / alpha = 1.78.  Everything below is computed by the CPU oracle
(float64 NumPy) from inputs drawn by the seeded generators; nothing comes from the GPU path.

Stored (at 2048 seeded mesh cells and 2048 seeded particles):
* delta of the CIC deposit (Sec. III A, Eq. CIC) at the sampled cells, and its sample checksum;
* lam, eps = <|S|> (Eq. normres) and the normalised residuals of the iterates u0, u1, u2 of the
  FFT-relaxation (Sec. III B, Eq. FFTrelax with the w-split of Sec. III C) from the linear guess;
* u2 (two updates) at the sampled cells;
* the force g = -(c/H0)^2 grad phi (Eq. FullDGP1, Sec. III A) with u = u2, interpolated with the
  CIC weights at the sampled particles, and the particles' float32 position and velocity after one
  kick-drift step (dlna = 0.005).

Run from the repository root:  python tests/golden/make_c4_512.py   (about 10 minutes, ~25 GB).
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import field as fld, pm, cosmology as cos  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402

N, BOX, SEED, OM0, A = 512, 1024.0, 4, 0.27, 0.5
RNL, DLNA, NSAMP = 1.78, 0.005, 2048
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_512_fixed2.json")


def log(*a):
    print("[%7.1f s]" % (time.time() - T0), *a, flush=True)


def main():
    pos, psi = inputs.zeldovich_load(N, BOX, SEED, dtype=np.float32)
    c = cos.coefficients(OM0, A)
    vel = (A * A * c.E * cos.omega_m_of_a(OM0, A) ** 0.55 * psi).astype(np.float32)
    del psi
    log("load built", pos.shape)
    _, delta = pm.deposit(pos, N, BOX)
    log("deposit done")
    cells = inputs.random_cells(N, NSAMP, 45)
    parts = np.sort(np.random.default_rng(46).choice(pos.shape[1], NSAMP, replace=False))
    prm = fld.SolveParams.from_cosmology(OM0, A)
    _, sk, _ = fld.source(delta, BOX, prm)
    ulin = fld.linear_solution(sk, BOX, prm)
    del sk
    lam = RNL * prm.alpha / float(np.max(np.abs(ulin)))
    del ulin
    log("lam", lam)
    prm = prm.with_(lam=lam, tol=0.0)
    u2, info = fld.solve(delta, BOX, prm, fixed_iters=2)
    log("two updates", info.history)
    assert info.history[0] > info.history[1] > info.history[2]
    force, _ = pm.pm_forces(delta, u2, pos[:, parts], BOX, prm, OM0, A)
    log("forces")
    x1, v1 = pm.kick_drift(pos[:, parts], vel[:, parts], force, A, DLNA, OM0, BOX)
    d_flat = delta.ravel()
    rec = {
        "_comment": __doc__.strip().splitlines()[0],
        "recipe": {"n": N, "box": BOX, "seed": SEED, "particles_dtype": "float32", "omega_m0": OM0, "a": A,
                   "r_nl": RNL, "w": 1.0 / 3.0, "dlna": DLNA, "cells_seed": 45, "particles_seed": 46,
                   "velocity": "a^2 E(a) Omega_m(a)^0.55 Psi, rounded to float32"},
        "lam": lam,
        "eps": info.eps,
        "history": info.history,
        "delta_checksum": {"sum_abs": float(np.sum(np.abs(d_flat))), "sum_sq": float(np.sum(d_flat * d_flat))},
        "cells": cells.tolist(),
        "delta": d_flat[cells].tolist(),
        "u2": u2.ravel()[cells].tolist(),
        "particles": parts.tolist(),
        "force": force.tolist(),
        "pos1": x1.astype(np.float64).tolist(),
        "vel1": v1.astype(np.float64).tolist(),
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
    log("wrote", OUT)


if __name__ == "__main__":
    T0 = time.time()
    main()
