"""ctypes declarations of the libdgp C-ABI (include/dgp.h).  Argument marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DGP_LIB_PATH") or os.path.join(HERE, "libdgp.so")

DGP_OK, DGP_NOT_CONVERGED, DGP_BAD_POINTS = 0, 1, 2
DGP_E_INVALID, DGP_E_NOMEM, DGP_E_HIP, DGP_E_UNSUPPORTED = -1, -2, -3, -4
DGP_FP64, DGP_FP32 = 0, 1
DGP_INIT_LINEAR, DGP_INIT_ZERO, DGP_INIT_WARM = 0, 1, 2
DGP_FORCE_NLDGP, DGP_FORCE_LDGP, DGP_FORCE_GRH, DGP_FORCE_GR = 0, 1, 2, 3

EXPORTS = (
    "dgp_params_init", "dgp_plan_create", "dgp_plan_create_ws", "dgp_workspace_bytes", "dgp_plan_destroy",
    "dgp_plan_device_bytes",
    "dgp_deposit", "dgp_solve_field", "dgp_pm_forces", "dgp_step", "dgp_solve_field_backward",
    "dgp_deposit_backward", "dgp_deposit_noalloc", "dgp_interp", "dgp_interp_backward", "dgp_power_spectrum", "dgp_power_spectrum_backward",
    "dgp_fft_forward", "dgp_fft_inverse", "dgp_timing_enable", "dgp_timing_classes", "dgp_timing_read",
    "dgp_run", "dgp_solve_history", "dgp_diagnostics", "dgp_last_error",
)
T_CLASSES = {"axis1_fwd": 0, "fanout": 1, "axis1_inv": 2, "relax": 3, "finalize": 4, "setup": 5,
             "deposit": 6, "forces": 7, "interp_kick": 8}
T_FP32_OFFSET = 16


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "omega_m0", "a", "E", "eta", "alpha", "beta", "A", "gamma", "c2", "kappa",
        "lambda_", "w", "omega_relax", "tol")] + [(n, ctypes.c_int) for n in (
            "max_iter", "init", "nonlocal_", "force_mode", "check_every", "spherical")]


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("status", "iters", "passes", "passes_fp64")] + [
        (n, ctypes.c_double) for n in ("resid", "resid_min", "eps", "bad_fraction", "mean_u", "ms_total")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

vp = ctypes.c_void_p
P = ctypes.POINTER


def load():
    """Load libdgp.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdgp.so is not built (%s); run `python -m paper_0906_4548_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "dgp_params_init": (ctypes.c_int, [P(Params), ctypes.c_double, ctypes.c_double]),
        "dgp_plan_create": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]),
        "dgp_plan_destroy": (ctypes.c_int, [vp]),
        "dgp_plan_device_bytes": (ctypes.c_size_t, [vp]),
        "dgp_plan_create_ws": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, vp,
                                              ctypes.c_size_t]),
        "dgp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "dgp_deposit": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_longlong, vp, vp, vp]),
        "dgp_solve_field": (ctypes.c_int, [vp, P(Params), vp, vp, vp, P(Info), vp]),
        "dgp_pm_forces": (ctypes.c_int, [vp, P(Params), vp, vp, vp, ctypes.c_int, ctypes.c_longlong, vp, vp, vp]),
        "dgp_step": (ctypes.c_int, [vp, P(Params), vp, vp, ctypes.c_int, ctypes.c_longlong, ctypes.c_double, vp,
                                    P(Info), vp]),
        "dgp_solve_field_backward": (ctypes.c_int, [vp, P(Params), vp, vp, vp, vp, P(Info), vp]),
        "dgp_deposit_backward": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_longlong, vp, vp, vp]),
        "dgp_deposit_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, vp, ctypes.c_int, ctypes.c_longlong, vp,
                                               vp, vp]),
        "dgp_interp": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_longlong, vp, vp]),
        "dgp_interp_backward": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_longlong, vp, vp, vp,
                                               vp]),
        "dgp_power_spectrum": (ctypes.c_int, [vp, P(Params), vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "dgp_power_spectrum_backward": (ctypes.c_int, [vp, P(Params), vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "dgp_fft_forward": (ctypes.c_int, [vp, vp, vp, vp]),
        "dgp_fft_inverse": (ctypes.c_int, [vp, vp, vp, vp]),
        "dgp_timing_enable": (ctypes.c_int, [vp, ctypes.c_int]),
        "dgp_timing_classes": (ctypes.c_int, [vp, ctypes.c_uint]),
        "dgp_run": (ctypes.c_int, [vp, ctypes.POINTER(Params), vp, vp, ctypes.c_int, ctypes.c_longlong,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double, vp,
                                   ctypes.POINTER(Info), vp]),
        "dgp_solve_history": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int]),
        "dgp_diagnostics": (ctypes.c_int, [vp, P(Params), vp, vp, vp, vp, vp, ctypes.c_int, vp]),
        "dgp_timing_read": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_longlong)]),
        "dgp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DGPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libdgp error %d: %s" % (code, msg))
        self.code = code


def check(code):
    """Raise on a negative status; return warnings (>= 0) unchanged."""
    if code < 0:
        raise DGPError(code, load().dgp_last_error().decode())
    return code
