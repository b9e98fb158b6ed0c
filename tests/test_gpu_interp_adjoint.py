"""CIC interpolation and its adjoint (dgp_interp, dgp_interp_backward, CICInterp) against the oracle.

Sec. III A: forces are interpolated with the deposit's assignment function (Eq. CIC).  The
adjoint gives dL/dpos (a gather with the dW/dx weights) and dL/dmesh (the transposed scatter,
summed in fixed point so that it has the same bits in any particle order).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import pm, adjoint  # noqa: E402
from paper_0906_4548_amd import inputs  # noqa: E402
from tests.gpu_common import to_dev, rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def dgp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_4548_amd import dgp as mod
    mod._lib.load()
    return mod


def say(*a):
    print(*a, flush=True)


def _case(n, box, npart, seed, nc=3, straddle=False):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(3, npart))
    if straddle:   # particles within a cell of the periodic boundary (their stencils wrap)
        pos[:, : npart // 2] = np.mod(rng.uniform(-box / n, box / n, size=(3, npart // 2)), box)
    mesh = rng.standard_normal((nc, n, n, n))
    gout = rng.standard_normal((nc, npart))
    return pos, mesh, gout


@pytest.mark.parametrize("case", [
    dict(n=16, npart=1000, nc=3, fp32=False),
    dict(n=16, npart=777, nc=1, fp32=False, straddle=True),     # ragged chunk, wrapped stencils
    dict(n=32, npart=3000, nc=2, fp32=True),
    dict(n=8, npart=1, nc=3, fp32=False),                         # a single particle
    dict(n=32, npart=32 ** 3, nc=3, fp32=False, zel=True),       # a coherent Zel'dovich load (binned path)
])
def test_interp_and_adjoint_match_oracle(dgp, case):
    say("interp adjoint", case)
    n, npart, nc = case["n"], case["npart"], case["nc"]
    box = 2.0 * n
    pos, mesh, gout = _case(n, box, npart, 100 + n + nc, nc, case.get("straddle", False))
    if case.get("zel"):
        pos, _ = inputs.zeldovich_load(n, box, 19, block=8)
    if case["fp32"]:
        pos = pos.astype(np.float32)
    out_ref = pm.cic_interpolate(mesh, pos, box)
    gpos_ref, gmesh_ref = adjoint.interp_backward(mesh, pos, gout, box)
    with dgp.Plan(n, box) as plan:
        tp = to_dev(pos, torch.float32 if case["fp32"] else torch.float64)
        out = torch.zeros((nc, npart), dtype=torch.float64, device="cuda")
        plan.interp(to_dev(mesh), tp, out)
        gpos = torch.zeros((3, npart), dtype=torch.float64, device="cuda")
        gmesh = torch.zeros((nc, n ** 3), dtype=torch.float64, device="cuda")
        plan.interp_backward(to_dev(mesh), tp, to_dev(gout), gpos, gmesh)
        torch.cuda.synchronize()
        assert rel_l2(out.cpu().numpy(), out_ref) <= 1e-13
        assert rel_l2(gpos.cpu().numpy(), gpos_ref) <= 1e-12
        assert rel_l2(gmesh.cpu().numpy().reshape(gmesh_ref.shape), gmesh_ref) <= 1e-12
        # only one of the two outputs
        gm2 = torch.zeros_like(gmesh)
        plan.interp_backward(None, tp, to_dev(gout), None, gm2)
        assert torch.equal(gm2, gmesh)


def test_mesh_adjoint_is_order_independent(dgp):
    """The fixed-point scatter gives the same bits for any particle order."""
    say("interp adjoint order")
    n, box, npart = 32, 64.0, 20000
    pos, mesh, gout = _case(n, box, npart, 7)
    perm = np.random.default_rng(8).permutation(npart)
    with dgp.Plan(n, box) as plan:
        outs = []
        for p in (None, perm):
            pp = pos if p is None else pos[:, p]
            gg = gout if p is None else gout[:, p]
            gm = torch.zeros((3, n ** 3), dtype=torch.float64, device="cuda")
            plan.interp_backward(None, to_dev(pp), to_dev(gg), None, gm)
            outs.append(gm.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])


def test_interp_adjoint_against_central_fd(dgp):
    """Central differences (step 1e-4 Mpc/h) of L = <g, interp(mesh, x)> in x, for particles at
    least 1e-3 cell away from every grid plane (the CIC weights are piecewise linear), and the
    exact linearity of L in the mesh (a random mesh direction)."""
    say("interp adjoint fd")
    n, box, npart = 16, 32.0, 400
    pos, mesh, gout = _case(n, box, npart, 9)
    s = pos * n / box
    ok = np.all(np.abs(s - np.round(s)) > 1e-3, axis=0)
    idx = np.flatnonzero(ok)[:64]
    h = 1e-4
    with dgp.Plan(n, box) as plan:
        tm, tg = to_dev(mesh), to_dev(gout)
        gpos = torch.zeros((3, npart), dtype=torch.float64, device="cuda")
        gmesh = torch.zeros((3, n ** 3), dtype=torch.float64, device="cuda")
        plan.interp_backward(tm, to_dev(pos), tg, gpos, gmesh)
        gpos = gpos.cpu().numpy()

        def loss(p, m=tm):
            out = torch.zeros((3, npart), dtype=torch.float64, device="cuda")
            plan.interp(m, to_dev(p), out)
            return float(torch.sum(out * tg))

        rng = np.random.default_rng(10)
        for k, p in enumerate(idx):
            d = int(rng.integers(3))
            q1, q2 = pos.copy(), pos.copy()
            q1[d, p] += h
            q2[d, p] -= h
            fd = (loss(q1) - loss(q2)) / (2 * h)
            assert abs(fd - gpos[d, p]) <= 1e-6 * max(abs(fd), abs(gpos[d, p])), (k, fd, gpos[d, p])
        dm = np.random.default_rng(11).standard_normal(mesh.shape)
        fd_m = (loss(pos, to_dev(mesh + dm)) - loss(pos, to_dev(mesh - dm))) / 2.0
        an_m = float(np.sum(dm.reshape(3, -1) * gmesh.cpu().numpy()))
        assert abs(fd_m - an_m) <= 1e-10 * abs(an_m)


def test_cic_interp_autograd(dgp):
    """CICInterp in an autograd graph: gradients with respect to both the mesh and positions."""
    say("interp autograd")
    from paper_0906_4548_amd.autograd import CICInterp
    n, box, npart = 16, 32.0, 500
    pos, mesh, gout = _case(n, box, npart, 12)
    gpos_ref, gmesh_ref = adjoint.interp_backward(mesh, pos, gout, box)
    with dgp.Plan(n, box) as plan:
        tm = to_dev(mesh.reshape(3, -1)).requires_grad_(True)
        tp = to_dev(pos).requires_grad_(True)
        out = CICInterp.apply(tm, tp, plan)
        torch.sum(out * to_dev(gout)).backward()
        assert rel_l2(tp.grad.cpu().numpy(), gpos_ref) <= 1e-12
        assert rel_l2(tm.grad.cpu().numpy().reshape(gmesh_ref.shape), gmesh_ref) <= 1e-12


def test_interp_backward_argument_errors(dgp):
    say("interp adjoint errors")
    n, box = 8, 16.0
    with dgp.Plan(n, box) as plan:
        pos = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
        g = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
        with pytest.raises(dgp._lib.DGPError) as e:
            plan.interp_backward(None, pos, g, None, None)
        assert e.value.code == -1
        with pytest.raises(dgp._lib.DGPError) as e:
            plan.interp_backward(None, pos, g, torch.zeros_like(g), None)
        assert e.value.code == -1
        # a non-finite gradient makes the mesh adjoint NaN (the call is asynchronous)
        gm = torch.zeros((3, n ** 3), dtype=torch.float64, device="cuda")
        g[1, 2] = float("inf")
        plan.interp_backward(None, pos, g, None, gm)
        assert bool(torch.all(torch.isnan(gm)))
