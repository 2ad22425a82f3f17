"""ctypes binding of libcurldiv (include/curldiv.h): argument marshalling only.

Every function here forwards to the C entry point of the same name.  Device
vectors are passed as raw device pointers (for example ``tensor.data_ptr()``
of a CUDA/HIP torch tensor) and the stream as a ``hipStream_t`` integer (for
example ``torch.cuda.current_stream().cuda_stream``).  The library must have
been built (``paper_1805_10058_amd/build.py``); importing this module without
it raises an error instead of falling back to anything else.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcurldiv.so")

CD_OK = 0
CD_NOT_CONVERGED = 1
CD_EINVAL = -1
CD_ENOMEM = -2
CD_EBREAKDOWN = -3
CD_EHIP = -4
CD_EAGAIN = -5
CD_ENOTFOUND = -6

CD_METHOD_PMIM = 0
CD_METHOD_PWL = 1
CD_METHOD_MIM = 2
CD_METHOD_CG = 3
CD_XFER_KNOT = 0
CD_XFER_PAPER = 1
CD_BOUNDS_LANCZOS = 0
CD_BOUNDS_SYMBOL = 1
CD_APPLY3D_AUTO = 0
CD_APPLY3D_MARCH = 1
CD_APPLY3D_SHORT = 2
CD_APPLY3D_GROUP = 3
CD_FP64 = 0
CD_MIXED_FP32 = 1


class cd_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


class cd_options(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("transfer", ctypes.c_int), ("precision", ctypes.c_int),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int), ("coarse_max_dofs", ctypes.c_int),
                ("cheb_degree", ctypes.c_int), ("cheb_ratio", ctypes.c_double), ("lanczos_steps", ctypes.c_int),
                ("krylov_steps", ctypes.c_int), ("graphs", ctypes.c_int), ("cheb_degree_coarse", ctypes.c_int),
                ("apply_x1_chunk", ctypes.c_int),
                ("eig_bounds", ctypes.c_int),
                ("bound_safety", ctypes.c_double),
                ("apply3d_kernel", ctypes.c_int)]


class cd_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class cd_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("kappa_estimate", ctypes.c_double)]


class cd_server_options(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int), ("num_streams", ctypes.c_int)]


class cd_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("result", cd_result), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("footprint_bytes", ctypes.c_size_t)]


# name -> (restype, argtypes); the exported symbol set of include/curldiv.h
_P = ctypes.c_void_p
_I = ctypes.c_int
SIGNATURES = {
    "cd_default_options": (None, [ctypes.POINTER(cd_options)]),
    "cd_num_dofs": (ctypes.c_size_t, [ctypes.POINTER(cd_problem)]),
    "cd_validate": (_I, [ctypes.POINTER(cd_problem), ctypes.POINTER(cd_options)]),
    "cd_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(cd_problem), ctypes.POINTER(cd_options)]),
    "cd_get_smoother": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "cd_graph_launches": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "cd_symbol_bound": (ctypes.c_int, [ctypes.POINTER(cd_problem), ctypes.POINTER(cd_options), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double)]),
    "cd_solver_create": (_I, [ctypes.POINTER(cd_problem), ctypes.POINTER(cd_options), _P, ctypes.POINTER(_P)]),
    "cd_solver_destroy": (None, [_P]),
    "cd_solve": (_I, [_P, _P, _P, ctypes.POINTER(cd_result)]),
    "cd_num_levels": (_I, [_P]),
    "cd_solver_device_bytes": (ctypes.c_size_t, [_P]),
    "cd_level_shape": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t)]),
    "cd_get_matrix": (_I, [_P, _I, _I, ctypes.c_char, ctypes.POINTER(ctypes.c_double)]),
    "cd_get_lambda": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double)]),
    "cd_apply": (_I, [_P, _I, _P, _P]),
    "cd_apply_f32": (_I, [_P, _I, _P, _P]),
    "cd_smooth": (_I, [_P, _I, _P, _P, _P]),
    "cd_restrict": (_I, [_P, _I, _P, _P]),
    "cd_prolong_add": (_I, [_P, _I, _P, _P]),
    "cd_tsolve": (_I, [_P, _P, _P]),
    "cd_smooth_f32": (_I, [_P, _I, _P, _P, _P]),
    "cd_restrict_f32": (_I, [_P, _I, _P, _P]),
    "cd_prolong_add_f32": (_I, [_P, _I, _P, _P]),
    "cd_tsolve_f32": (_I, [_P, _P, _P]),
    "cd_tsolve_noalloc": (_I, [_P, _P, _P]),
    "cd_coarse_solve": (_I, [_P, _P, _P]),
    "cd_load_vector": (_I, [_P, _P]),
    "cd_l2_error": (_I, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "cd_precondition": (_I, [_P, _P, _P]),
    "cd_profile_enable": (_I, [_P, _I]),
    "cd_profile_read": (_I, [_P, _I, _I, ctypes.POINTER(cd_kernel_stats)]),
    "cd_profile_read_smoother": (_I, [_P, _I, _I, ctypes.POINTER(cd_kernel_stats)]),
    "cd_profile_read_tsolve": (_I, [_P, _I, ctypes.POINTER(cd_kernel_stats)]),
    "cd_server_default_options": (None, [ctypes.POINTER(cd_server_options)]),
    "cd_server_create": (_I, [ctypes.POINTER(cd_server_options), ctypes.POINTER(_P)]),
    "cd_server_submit": (_I, [_P, ctypes.POINTER(cd_problem), ctypes.POINTER(cd_options), _P, _P,
                              ctypes.POINTER(ctypes.c_uint64)]),
    "cd_server_step": (_I, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "cd_server_poll": (_I, [_P, ctypes.POINTER(cd_completion), _I, ctypes.POINTER(ctypes.c_int)]),
    "cd_server_destroy": (None, [_P]),
    "cd_status_string": (ctypes.c_char_p, [_I]),
    "cd_last_error": (ctypes.c_char_p, []),
}


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1805_10058_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


class CurldivError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def check(rc, allow=(CD_OK,)):
    if rc not in allow:
        raise CurldivError(rc, lib().cd_last_error().decode() or lib().cd_status_string(rc).decode())
    return rc


def problem(dim, degree, n, alpha, beta):
    ns = list(n) if hasattr(n, "__len__") else [n] * dim
    ns = ns + [1] * (3 - len(ns))
    return cd_problem(dim, degree, (ctypes.c_int * 3)(*ns), float(alpha), float(beta))


def options(**kw):
    o = cd_options()
    lib().cd_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def num_dofs(prob):
    return lib().cd_num_dofs(ctypes.byref(prob))


def footprint_bytes(prob, opt):
    return lib().cd_footprint_bytes(ctypes.byref(prob), ctypes.byref(opt))


def validate(prob, opt):
    return lib().cd_validate(ctypes.byref(prob), ctypes.byref(opt))


def symbol_bound(prob, opt, level):
    lam = ctypes.c_double()
    check(lib().cd_symbol_bound(ctypes.byref(prob), ctypes.byref(opt), int(level), ctypes.byref(lam)))
    return lam.value


class Solver:
    """Owner of a cd_solver handle; methods forward to the C entry points."""

    def __init__(self, prob, opt, stream=0):
        self._h = ctypes.c_void_p()
        self.prob, self.opt = prob, opt
        check(lib().cd_solver_create(ctypes.byref(prob), ctypes.byref(opt), ctypes.c_void_p(stream),
                                     ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().cd_solver_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def solve(self, b_ptr, x_ptr):
        res = cd_result()
        rc = lib().cd_solve(self._h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), ctypes.byref(res))
        check(rc, allow=(CD_OK, CD_NOT_CONVERGED))
        return res

    def device_bytes(self):
        return lib().cd_solver_device_bytes(self._h)

    def num_levels(self):
        return lib().cd_num_levels(self._h)

    def level_shape(self, level):
        m = (ctypes.c_int * 3)()
        n = ctypes.c_size_t()
        check(lib().cd_level_shape(self._h, level, m, ctypes.byref(n)))
        return tuple(m), n.value

    def get_matrix(self, level, axis, which, rows, cols):
        buf = (ctypes.c_double * (rows * cols))()
        check(lib().cd_get_matrix(self._h, level, axis, which.encode(), buf))
        return buf

    def get_smoother(self, level):
        deg, lo, hi = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        check(lib().cd_get_smoother(self._h, level, ctypes.byref(deg), ctypes.byref(lo), ctypes.byref(hi)))
        return deg.value, lo.value, hi.value

    def coarse_degree(self):
        """The Chebyshev degree of the levels below the finest (None with one smoothed level)."""
        return self.get_smoother(1)[0] if self.num_levels() > 2 else None

    def graph_launches(self):
        k, n = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().cd_graph_launches(self._h, ctypes.byref(k), ctypes.byref(n)))
        return k.value, n.value

    def get_lambda(self, level):
        v = ctypes.c_double()
        check(lib().cd_get_lambda(self._h, level, ctypes.byref(v)))
        return v.value

    def apply(self, level, x_ptr, y_ptr):
        check(lib().cd_apply(self._h, level, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)))

    def apply_f32(self, level, x_ptr, y_ptr):
        check(lib().cd_apply_f32(self._h, level, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)))

    def smooth(self, level, b_ptr, x_in_ptr, x_out_ptr):
        check(lib().cd_smooth(self._h, level, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_in_ptr),
                              ctypes.c_void_p(x_out_ptr)))

    def restrict(self, level, rf_ptr, rc_ptr):
        check(lib().cd_restrict(self._h, level, ctypes.c_void_p(rf_ptr), ctypes.c_void_p(rc_ptr)))

    def prolong_add(self, level, ec_ptr, xf_ptr):
        check(lib().cd_prolong_add(self._h, level, ctypes.c_void_p(ec_ptr), ctypes.c_void_p(xf_ptr)))

    def smooth_f32(self, level, b_ptr, x_in_ptr, x_out_ptr):
        check(lib().cd_smooth_f32(self._h, level, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_in_ptr),
                                  ctypes.c_void_p(x_out_ptr)))

    def restrict_f32(self, level, rf_ptr, rc_ptr):
        check(lib().cd_restrict_f32(self._h, level, ctypes.c_void_p(rf_ptr), ctypes.c_void_p(rc_ptr)))

    def prolong_add_f32(self, level, ec_ptr, xf_ptr):
        check(lib().cd_prolong_add_f32(self._h, level, ctypes.c_void_p(ec_ptr), ctypes.c_void_p(xf_ptr)))

    def tsolve_f32(self, v_ptr, z_ptr):
        check(lib().cd_tsolve_f32(self._h, ctypes.c_void_p(v_ptr), ctypes.c_void_p(z_ptr)))

    def tsolve(self, v_ptr, z_ptr):
        check(lib().cd_tsolve(self._h, ctypes.c_void_p(v_ptr), ctypes.c_void_p(z_ptr)))

    def tsolve_noalloc(self, v_ptr, z_ptr):
        check(lib().cd_tsolve_noalloc(self._h, ctypes.c_void_p(v_ptr), ctypes.c_void_p(z_ptr)))

    def load_vector(self, b_ptr):
        check(lib().cd_load_vector(self._h, ctypes.c_void_p(b_ptr)))

    def l2_error(self, x_ptr):
        e = ctypes.c_double()
        check(lib().cd_l2_error(self._h, ctypes.c_void_p(x_ptr), ctypes.byref(e)))
        return e.value

    def coarse_solve(self, r_ptr, z_ptr):
        check(lib().cd_coarse_solve(self._h, ctypes.c_void_p(r_ptr), ctypes.c_void_p(z_ptr)))

    def profile_enable(self, on=True, period=1):
        """Live timing of operator applies; during solves every `period`-th
        outer iteration is timed."""
        check(lib().cd_profile_enable(self._h, max(int(period), 1) if on else 0))

    def profile_read(self, level, fp32):
        st = cd_kernel_stats()
        check(lib().cd_profile_read(self._h, level, 1 if fp32 else 0, ctypes.byref(st)))
        return st

    def profile_read_smoother(self, level, fp32):
        st = cd_kernel_stats()
        check(lib().cd_profile_read_smoother(self._h, level, 1 if fp32 else 0, ctypes.byref(st)))
        return st

    def profile_read_tsolve(self, fp32=False):
        st = cd_kernel_stats()
        check(lib().cd_profile_read_tsolve(self._h, 1 if fp32 else 0, ctypes.byref(st)))
        return st

    def precondition(self, r_ptr, z_ptr):
        check(lib().cd_precondition(self._h, ctypes.c_void_p(r_ptr), ctypes.c_void_p(z_ptr)))


class Server:
    """Owner of a cd_server handle; methods forward to the C entry points."""

    def __init__(self, hbm_budget_bytes=0, max_active=0, num_streams=0):
        o = cd_server_options()
        lib().cd_server_default_options(ctypes.byref(o))
        if hbm_budget_bytes:
            o.hbm_budget_bytes = hbm_budget_bytes
        if max_active:
            o.max_active = max_active
        if num_streams:
            o.num_streams = num_streams
        self._h = ctypes.c_void_p()
        check(lib().cd_server_create(ctypes.byref(o), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().cd_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, prob, opt, b_ptr, x_ptr):
        t = ctypes.c_uint64()
        check(lib().cd_server_submit(self._h, ctypes.byref(prob), ctypes.byref(opt), ctypes.c_void_p(b_ptr),
                                     ctypes.c_void_p(x_ptr), ctypes.byref(t)))
        return t.value

    def step(self):
        a, q = ctypes.c_int(), ctypes.c_int()
        check(lib().cd_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, max_n=256):
        buf = (cd_completion * max_n)()
        n = ctypes.c_int()
        check(lib().cd_server_poll(self._h, buf, max_n, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]
