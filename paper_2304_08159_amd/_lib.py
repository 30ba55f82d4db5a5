"""ctypes binding of libwl.so (argument marshalling only).

Every computation happens in the HIP library; this module converts Python
arguments into the C ABI declared in include/wl.h and hands torch device
pointers and the current HIP stream to it.  There is no fallback: when the
library is missing or no GPU is present, the calls raise.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwl.so")

WL_OK = 0
WL_ERR_INVALID_ARG, WL_ERR_NOT_CONVERGED, WL_ERR_NONFINITE = -1, -3, -4
STATUS = {
    0: "WL_OK", -1: "WL_ERR_INVALID_ARG", -2: "WL_ERR_OUT_OF_MEMORY",
    -3: "WL_ERR_NOT_CONVERGED", -4: "WL_ERR_NONFINITE", -5: "WL_ERR_HIP", -6: "WL_ERR_STATE",
}
WL_FP32, WL_FP64, WL_MIXED = 0, 1, 2
STOP_DIVERGENCE, STOP_RELATIVE = 0, 1
SMOOTH_JACOBI, SMOOTH_CG = 0, 1
PERIODIC, INFLOW, OUTFLOW, WALL = 0, 1, 2, 3

FIELD_U0, FIELD_U1, FIELD_U2, FIELD_P, FIELD_UOUT = 0, 1, 2, 3, 4
FIELD_L0, FIELD_MU0_0, FIELD_MU1N, FIELD_SIGMA = 5, 8, 11, 20

# Every symbol include/wl.h declares.
EXPORTS = (
    "wl_sim_footprint", "wl_sim_create", "wl_sim_destroy", "wl_set_field", "wl_get_field",
    "wl_set_time", "wl_state_size", "wl_get_state", "wl_set_state", "wl_step", "wl_run",
    "wl_drag", "wl_tape_record", "wl_step_adjoint",
    "wl_poisson_footprint", "wl_poisson_create",
    "wl_poisson_solve", "wl_poisson_destroy", "wl_poisson_batch_footprint",
    "wl_poisson_batch_solve", "wl_poisson_batch_solve_noalloc", "wl_ns_batch_footprint",
    "wl_ns_batch_run", "wl_body_coeffs",
    "wl_set_graphs", "wl_set_fused_sweeps", "wl_set_smoother",
    "wl_profile_enable",
    "wl_profile_reset",
    "wl_profile_read", "wl_last_error", "wl_version",
)
PROF = dict(smooth_fine=0, smooth_norm=1, prolong_fine=2, restrict_fine=3, momentum=4,
            divergence=5, project=6, norm_fine=7, pair_fine=8, pair_prolong_fine=9)


class WlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("centre", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("eps", ctypes.c_double),
                ("radius2", ctypes.c_double), ("velocity", ctypes.c_double * 3),
                ("amplitude", ctypes.c_double * 3), ("omega", ctypes.c_double),
                ("spin", ctypes.c_double * 3)]


def body_kind(body):
    """wl_body.kind of a body dict: {"kind": "torus"} selects 2, else a sphere (1)."""
    return 2 if body.get("kind", "sphere") == "torus" else 1


def fill_body(b, body, ndim, eps=1.0):
    """Fill a Body from a dict: centre, radius, optional kind / radius2 / eps
    and motion (velocity, amplitude, omega; spin as a 3-vector, or a scalar
    about z)."""
    b.kind = body_kind(body)
    b.radius2 = float(body.get("radius2", 0.0))
    c = list(body["centre"]) + [0.0] * (3 - ndim)
    v = list(body.get("velocity", (0.0,) * ndim)) + [0.0] * (3 - ndim)
    a = list(body.get("amplitude", (0.0,) * ndim)) + [0.0] * (3 - ndim)
    sp = body.get("spin", 0.0)
    sp = [0.0, 0.0, float(sp)] if not hasattr(sp, "__len__") else list(sp) + [0.0] * (3 - len(sp))
    for i in range(3):
        b.centre[i] = float(c[i])
        b.velocity[i] = float(v[i])
        b.amplitude[i] = float(a[i])
        b.spin[i] = float(sp[i])
    b.omega = float(body.get("omega", 0.0))
    b.radius = float(body["radius"])
    b.eps = float(body.get("eps", eps))


class SimDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3),
                ("U", ctypes.c_double * 3), ("nu", ctypes.c_double), ("body", Body),
                ("prec", ctypes.c_int), ("mg_levels", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_vcycles", ctypes.c_int), ("inner_vcycles", ctypes.c_int),
                ("cfl", ctypes.c_double), ("tape_steps", ctypes.c_int),
                ("stop_rule", ctypes.c_int)]


class BatchRequest(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("periodic", ctypes.c_int * 3),
                ("coeffs", ctypes.c_void_p), ("x", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("max_vcycles", ctypes.c_int), ("mixed", ctypes.c_int)]


class BatchResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("vcycles", ctypes.c_int), ("rel_resid", ctypes.c_double)]


class NsRequest(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("bc_lo", ctypes.c_int * 3),
                ("bc_hi", ctypes.c_int * 3), ("U", ctypes.c_double * 3), ("nu", ctypes.c_double),
                ("body", Body), ("tol", ctypes.c_double), ("max_vcycles", ctypes.c_int),
                ("steps", ctypes.c_int), ("cfl", ctypes.c_double), ("u", ctypes.c_void_p),
                ("uout", ctypes.c_void_p), ("p", ctypes.c_void_p)]


class NsResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("vcycles", ctypes.c_int), ("t", ctypes.c_double),
                ("dt", ctypes.c_double)]


class StepStats(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("t", ctypes.c_double),
                ("vcycles", ctypes.c_int * 2), ("resid", ctypes.c_double * 2),
                ("rel_resid", ctypes.c_double * 2)]


_lib = None


def load():
    """Load libwl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2304_08159_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ip3 = ctypes.POINTER(ctypes.c_int)
    sig = {
        "wl_sim_footprint": [ctypes.POINTER(SimDesc), ctypes.POINTER(sz)],
        "wl_sim_create": [ctypes.POINTER(SimDesc), vp, sz, vp, ctypes.POINTER(vp)],
        "wl_sim_destroy": [vp],
        "wl_set_field": [vp, i32, vp],
        "wl_get_field": [vp, i32, vp],
        "wl_set_time": [vp, f64],
        "wl_state_size": [vp, ctypes.POINTER(sz)],
        "wl_get_state": [vp, vp],
        "wl_set_state": [vp, vp],
        "wl_step": [vp, f64, ctypes.POINTER(StepStats)],
        "wl_run": [vp, i32, f64, ctypes.POINTER(StepStats), ctypes.POINTER(i32)],
        "wl_drag": [vp, ctypes.POINTER(f64)],
        "wl_tape_record": [vp, i32],
        "wl_step_adjoint": [vp, vp, vp, f64, vp, ctypes.POINTER(f64)],
        "wl_poisson_footprint": [i32, ip3, ip3, i32, i32, ctypes.POINTER(sz)],
        "wl_poisson_create": [i32, ip3, ip3, i32, i32, vp, sz, vp, ctypes.POINTER(vp)],
        "wl_poisson_solve": [vp, vp, vp, vp, f64, i32, ctypes.POINTER(i32), ctypes.POINTER(f64)],
        "wl_poisson_destroy": [vp],
        "wl_poisson_batch_footprint": [ctypes.POINTER(BatchRequest), i32, ctypes.POINTER(sz)],
        "wl_poisson_batch_solve": [ctypes.POINTER(BatchRequest), i32, vp, sz, vp,
                                   ctypes.POINTER(BatchResult)],
        "wl_poisson_batch_solve_noalloc": [ctypes.POINTER(BatchRequest), i32, vp,
                                           ctypes.POINTER(BatchResult)],
        "wl_ns_batch_footprint": [ctypes.POINTER(NsRequest), i32, ctypes.POINTER(sz)],
        "wl_ns_batch_run": [ctypes.POINTER(NsRequest), i32, vp, sz, vp, ctypes.POINTER(NsResult)],
        "wl_body_coeffs": [ctypes.POINTER(Body), i32, ip3, ip3, i32, vp, vp],
        "wl_set_graphs": [i32],
        "wl_set_fused_sweeps": [i32],
        "wl_set_smoother": [i32],
        "wl_profile_enable": [ctypes.c_uint],
        "wl_profile_reset": [],
        "wl_profile_read": [i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_longlong),
                            ctypes.POINTER(ctypes.c_longlong)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.wl_last_error.restype = ctypes.c_char_p
    lib.wl_last_error.argtypes = []
    lib.wl_version.restype = ctypes.c_char_p
    lib.wl_version.argtypes = []
    _lib = lib
    return lib


def check(status, allow=()):
    if status != WL_OK and status not in allow:
        raise WlError(status, load().wl_last_error().decode())
    return status
