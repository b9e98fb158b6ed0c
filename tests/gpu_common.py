"""Shared helpers of the GPU parity tests (inputs, oracle calls, tolerances)."""
import numpy as np
import torch

from oracle import field as fld
from oracle import cosmology as cos

OM0 = 0.27


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype).contiguous()


def oracle_params(a=0.5, **kw):
    return fld.SolveParams.from_cosmology(OM0, a, **kw)


def calibrate_lambda(delta, box, rnl, a=0.5):
    """lam such that lam * max|u_lin| / alpha = rnl (u_lin: linear solution from the oracle)."""
    prm = oracle_params(a)
    _, sk, _ = fld.source(delta, box, prm)
    ul = fld.linear_solution(sk, box, prm)
    return rnl * prm.alpha / np.max(np.abs(ul))


def gpu_params(dgp, a=0.5, **kw):
    return dgp.params(OM0, a, **kw)


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))
