"""Seeded input generators (shared by the oracle and the GPU path): host-only checks."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_0906_4548_amd import inputs  # noqa: E402


def test_blocked_order_is_a_permutation_into_compact_blocks():
    n, box, b = 16, 32.0, 4
    lat, psi_lat = inputs.zeldovich_load(n, box, 7)
    blk, psi_blk = inputs.zeldovich_load(n, box, 7, block=b)
    # same particles, reordered
    key = lambda x: np.lexsort(x)  # noqa: E731
    assert np.array_equal(lat[:, key(psi_lat)], blk[:, key(psi_blk)])
    # every run of b^3 particles is one Lagrangian block: lattice sites q = x - psi
    h = box / n
    q = np.rint((blk - psi_blk) / h - 0.5).astype(np.int64) % n
    for c in range(0, n ** 3, b ** 3):
        site = q[:, c:c + b ** 3]
        assert all(len(np.unique(site[d] // b)) == 1 for d in range(3))
        assert len({tuple(t) for t in site.T}) == b ** 3


def test_lattice_order_axis2_fastest():
    n, box = 8, 16.0
    x, psi = inputs.zeldovich_load(n, box, 3)
    q = np.rint((x - psi) / (box / n) - 0.5).astype(np.int64) % n
    idx = (q[0] * n + q[1]) * n + q[2]
    assert np.array_equal(idx, np.arange(n ** 3))
