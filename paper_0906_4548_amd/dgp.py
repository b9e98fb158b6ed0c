"""Python binding of libdgp with torch tensors (device memory and streams only).

Every function validates shapes / dtypes / devices, passes raw device pointers
and the current torch stream to the C-ABI of include/dgp.h, and raises on an
error status.  No arithmetic of the method happens here.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Params, Info, check

FP64, FP32 = _lib.DGP_FP64, _lib.DGP_FP32
INIT_LINEAR, INIT_ZERO, INIT_WARM = _lib.DGP_INIT_LINEAR, _lib.DGP_INIT_ZERO, _lib.DGP_INIT_WARM
FORCE_NLDGP, FORCE_LDGP, FORCE_GRH, FORCE_GR = (_lib.DGP_FORCE_NLDGP, _lib.DGP_FORCE_LDGP, _lib.DGP_FORCE_GRH,
                                              _lib.DGP_FORCE_GR)


def params(omega_m0=0.27, a=0.5, **overrides):
    """dgp_params filled by dgp_params_init, then overridden by keyword (``lam`` for lambda)."""
    p = Params()
    check(_lib.load().dgp_params_init(ctypes.byref(p), float(omega_m0), float(a)))
    for k, v in overrides.items():
        key = {"lam": "lambda_", "lambda": "lambda_", "nonlocal": "nonlocal_"}.get(k, k)
        if not hasattr(p, key):
            raise KeyError(k)
        setattr(p, key, v)
    return p


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def workspace_bytes(n, batch=1, precision=FP64, with_adjoint=False):
    """Device bytes a plan of these sizes uses (dgp_workspace_bytes); 0 for invalid sizes."""
    return int(_lib.load().dgp_workspace_bytes(int(n), int(batch), int(precision), 1 if with_adjoint else 0))


class Plan:
    """Workspace for an N^3 mesh of side ``box`` with ``batch`` fields in ``precision``.

    ``workspace``: optional caller-owned device buffer (a CUDA tensor of at least
    ``workspace_bytes(n, batch, precision)`` bytes, 256-byte aligned, as torch allocates); the
    plan then carves its device buffers from it (dgp_plan_create_ws) and keeps a reference."""

    def __init__(self, n, box, batch=1, precision=FP64, workspace=None):
        self.n, self.box, self.batch, self.precision = int(n), float(box), int(batch), int(precision)
        h = ctypes.c_void_p()
        self._ws = workspace
        if workspace is None:
            check(_lib.load().dgp_plan_create(ctypes.byref(h), self.n, self.batch, self.box, self.precision))
        else:
            nbytes = workspace.numel() * workspace.element_size()
            check(_lib.load().dgp_plan_create_ws(ctypes.byref(h), self.n, self.batch, self.box, self.precision,
                                                 _ptr(workspace, None, None, "workspace"), nbytes))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    @property
    def n3(self):
        return self.n ** 3

    def device_bytes(self):
        return int(_lib.load().dgp_plan_device_bytes(self.handle))

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().dgp_plan_destroy(self._h)
            self._h = None
        self._ws = None   # a caller workspace may be released once the plan is gone

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- entry points
    def deposit(self, pos, grid=None, delta=None):
        """CIC deposit of pos [3, np]; fills grid (int64 [N^3]) and/or delta (float64 [N^3])."""
        npart = pos.shape[-1]
        fp32 = 1 if pos.dtype == torch.float32 else 0
        _ptr(pos, None, 3 * npart, "pos")
        return check(_lib.load().dgp_deposit(self.handle, _ptr(pos), fp32, npart,
                                             _ptr(grid, torch.int64, self.n3, "grid"),
                                             _ptr(delta, torch.float64, self.n3, "delta"), _stream()))

    def solve_field(self, prm, delta, u_state, c_out=None):
        """Field solve; returns (status, [info dict per batch element])."""
        cnt = self.batch * self.n3
        infos = (Info * self.batch)()
        st = check(_lib.load().dgp_solve_field(self.handle, ctypes.byref(prm), _ptr(delta, torch.float64, cnt, "delta"),
                                               _ptr(u_state, torch.float64, cnt, "u_state"),
                                               _ptr(c_out, torch.float64, cnt, "c_out"), infos, _stream()))
        return st, [i.as_dict() for i in infos]

    def pm_forces(self, prm, delta, u_state, pos, force, phi_n=None):
        npart = pos.shape[-1]
        fp32 = 1 if pos.dtype == torch.float32 else 0
        return check(_lib.load().dgp_pm_forces(
            self.handle, ctypes.byref(prm), _ptr(delta, torch.float64, self.n3, "delta"),
            _ptr(u_state, torch.float64, self.n3, "u_state"), _ptr(pos, None, 3 * npart, "pos"), fp32, npart,
            _ptr(force, torch.float64, 3 * npart, "force"), _ptr(phi_n, torch.float64, self.n3, "phi_n"), _stream()))

    def step(self, prm, pos, vel, u_state, dlna):
        npart = pos.shape[-1]
        if vel.dtype != pos.dtype:
            raise TypeError("pos and vel must share a dtype")
        fp32 = 1 if pos.dtype == torch.float32 else 0
        infos = (Info * 1)()
        st = check(_lib.load().dgp_step(self.handle, ctypes.byref(prm), _ptr(pos, None, 3 * npart, "pos"),
                                        _ptr(vel, None, 3 * npart, "vel"), fp32, npart, float(dlna),
                                        _ptr(u_state, torch.float64, self.n3, "u_state"), infos, _stream()))
        return st, infos[0].as_dict()

    def run(self, prm, pos, vel, u_state, a_start, dlna, n_steps, a_switch):
        """dgp_run: n_steps PM steps from a_start (lDGP forces before a_switch, then the
        plan's solve with warm starts).  Returns (worst status, [info dict per step])."""
        npart = pos.shape[-1]
        if vel.dtype != pos.dtype:
            raise TypeError("pos and vel must share a dtype")
        fp32 = 1 if pos.dtype == torch.float32 else 0
        infos = (Info * max(1, int(n_steps)))()
        st = check(_lib.load().dgp_run(self.handle, ctypes.byref(prm), _ptr(pos, None, 3 * npart, "pos"),
                                       _ptr(vel, None, 3 * npart, "vel"), fp32, npart, float(a_start),
                                       float(dlna), int(n_steps), float(a_switch),
                                       _ptr(u_state, torch.float64, self.n3, "u_state"), infos, _stream()))
        return st, [infos[k].as_dict() for k in range(int(n_steps))]

    def history(self, b=0, cap=256):
        """(residual per pass, bad-point fraction per pass) of the last solve of element b."""
        r = (ctypes.c_double * cap)()
        f = (ctypes.c_double * cap)()
        m = check(_lib.load().dgp_solve_history(self.handle, int(b), r, f, int(cap)))
        return np.array(r[:m]), np.array(f[:m])

    def solve_field_backward(self, prm, delta, u_star, grad_u, grad_delta):
        cnt = self.batch * self.n3
        infos = (Info * self.batch)()
        st = check(_lib.load().dgp_solve_field_backward(
            self.handle, ctypes.byref(prm), _ptr(delta, torch.float64, cnt, "delta"),
            _ptr(u_star, torch.float64, cnt, "u_star"), _ptr(grad_u, torch.float64, cnt, "grad_u"),
            _ptr(grad_delta, torch.float64, cnt, "grad_delta"), infos, _stream()))
        return st, [i.as_dict() for i in infos]

    def deposit_backward(self, pos, grad_delta, grad_pos):
        npart = pos.shape[-1]
        fp32 = 1 if pos.dtype == torch.float32 else 0
        return check(_lib.load().dgp_deposit_backward(
            self.handle, _ptr(pos, None, 3 * npart, "pos"), fp32, npart,
            _ptr(grad_delta, torch.float64, self.n3, "grad_delta"),
            _ptr(grad_pos, torch.float64, 3 * npart, "grad_pos"), _stream()))

    def interp(self, mesh, pos, out):
        """CIC interpolation out [ncomp, np] of mesh [ncomp, N^3] (float64) at pos [3, np]."""
        npart = pos.shape[-1]
        nc = mesh.numel() // self.n3
        fp32 = 1 if pos.dtype == torch.float32 else 0
        return check(_lib.load().dgp_interp(
            self.handle, _ptr(mesh, torch.float64, nc * self.n3, "mesh"), nc, _ptr(pos, None, 3 * npart, "pos"), fp32,
            npart, _ptr(out, torch.float64, nc * npart, "out"), _stream()))

    def interp_backward(self, mesh, pos, grad_out, grad_pos=None, grad_mesh=None):
        """Adjoint of interp: grad_pos [3, np] and/or grad_mesh [ncomp, N^3] (float64) from
        grad_out [ncomp, np]; mesh is needed only for grad_pos."""
        npart = pos.shape[-1]
        nc = grad_out.numel() // npart
        fp32 = 1 if pos.dtype == torch.float32 else 0
        return check(_lib.load().dgp_interp_backward(
            self.handle, _ptr(mesh, torch.float64, nc * self.n3, "mesh"), nc, _ptr(pos, None, 3 * npart, "pos"), fp32,
            npart, _ptr(grad_out, torch.float64, nc * npart, "grad_out"),
            _ptr(grad_pos, torch.float64, 3 * npart, "grad_pos"),
            _ptr(grad_mesh, torch.float64, nc * self.n3, "grad_mesh"), _stream()))

    def power_spectrum(self, prm, field, of_c=False, nbins=64):
        """Returns (pk [batch, nbins] numpy, counts [nbins] numpy)."""
        pk = np.zeros((self.batch, nbins))
        cnt = np.zeros(nbins)
        check(_lib.load().dgp_power_spectrum(
            self.handle, ctypes.byref(prm), _ptr(field, torch.float64, self.batch * self.n3, "field"), int(bool(of_c)),
            nbins, pk.ctypes.data_as(ctypes.c_void_p), cnt.ctypes.data_as(ctypes.c_void_p), _stream()))
        return pk, cnt

    def diagnostics(self, prm, delta, u, nbins=64):
        """Diagnostics of a solved field u (Appendix, Eq. EllipticMatrix; Eqs. cdef, DGradC):
        returns (non-elliptic fraction [batch], P_c/P_m [batch, nbins], Delta_gradC [batch, nbins])
        as numpy arrays; P_c/P_m needs delta (None skips it)."""
        ne = np.zeros(self.batch)
        ratio = np.zeros((self.batch, nbins))
        dgc = np.zeros((self.batch, nbins))
        cnt = self.batch * self.n3
        dptr = _ptr(delta, torch.float64, cnt, "delta") if delta is not None else None
        check(_lib.load().dgp_diagnostics(
            self.handle, ctypes.byref(prm), dptr, _ptr(u, torch.float64, cnt, "u"),
            ne.ctypes.data_as(ctypes.c_void_p), ratio.ctypes.data_as(ctypes.c_void_p) if delta is not None else None,
            dgc.ctypes.data_as(ctypes.c_void_p), int(nbins), _stream()))
        return ne, (ratio if delta is not None else None), dgc

    def power_spectrum_backward(self, prm, field, grad_pk, grad_field, of_c=False):
        g = np.ascontiguousarray(grad_pk, dtype=np.float64).reshape(self.batch, -1)
        return check(_lib.load().dgp_power_spectrum_backward(
            self.handle, ctypes.byref(prm), _ptr(field, torch.float64, self.batch * self.n3, "field"),
            int(bool(of_c)), g.shape[1], g.ctypes.data_as(ctypes.c_void_p),
            _ptr(grad_field, torch.float64, self.batch * self.n3, "grad_field"), _stream()))

    def timing(self, on=True):
        """Enable (and reset) or disable live HIP-event timing of the plan's kernel classes."""
        check(_lib.load().dgp_timing_enable(self.handle, int(bool(on))))

    def timing_classes(self, names=None):
        """Time only the given classes (names as returned by timing_read, e.g. 'relax_fp32');
        None times every class."""
        mask = 0xFFFFFFFF
        if names is not None:
            mask = 0
            for nm in names:
                base, off = (nm[:-5], _lib.T_FP32_OFFSET) if nm.endswith("_fp32") else (nm, 0)
                mask |= 1 << (_lib.T_CLASSES[base] + off)
        check(_lib.load().dgp_timing_classes(self.handle, ctypes.c_uint(mask)))

    def timing_read(self):
        """{class name: (total ms, launches)} including float32 classes as '<name>_fp32'."""
        out = {}
        for name, cls in _lib.T_CLASSES.items():
            for suffix, off in (("", 0), ("_fp32", _lib.T_FP32_OFFSET)):
                ms = ctypes.c_double()
                cnt = ctypes.c_longlong()
                check(_lib.load().dgp_timing_read(self.handle, cls + off, ctypes.byref(ms), ctypes.byref(cnt)))
                if cnt.value:
                    out[name + suffix] = (ms.value, cnt.value)
        return out

    def fft_forward(self, field, spectrum):
        """spectrum: complex128 [batch, N/2+1, N, N] (half axis first)."""
        hs = self.batch * (self.n // 2 + 1) * self.n * self.n
        return check(_lib.load().dgp_fft_forward(self.handle, _ptr(field, torch.float64, self.batch * self.n3, "field"),
                                                 _ptr(spectrum, torch.complex128, hs, "spectrum"), _stream()))

    def fft_inverse(self, spectrum, field):
        hs = self.batch * (self.n // 2 + 1) * self.n * self.n
        return check(_lib.load().dgp_fft_inverse(self.handle, _ptr(spectrum, torch.complex128, hs, "spectrum"),
                                                 _ptr(field, torch.float64, self.batch * self.n3, "field"), _stream()))
