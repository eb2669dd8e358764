"""Thin ctypes binding of libridg (C ABI in include/ridg.h).

Argument marshalling only: every step of the prediction and correction runs in
the library's HIP kernels. PyTorch provides the device workspace and the stream.
The binding refuses to run when the shared library is missing: there is no
fallback path.
"""

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libridg.so")

RIDG_OK = 0
RIDG_E_INVAL = -1
RIDG_E_NOMEM = -2
RIDG_E_DEVICE = -3
RIDG_E_SINGULAR = -4
RIDG_E_NONFINITE = -5
RIDG_E_UNSUPPORTED = -6
RIDG_W_UNSTABLE = 1
RIDG_W_NOT_CONVERGED = 2

FLUX_CONST, FLUX_ROTATION, FLUX_AFFINE, FLUX_BURGERS = 0, 1, 2, 3
BASIS_P, BASIS_Q = 0, 1
ABI_VERSION = 3
FP64, FP32_REFINE = 0, 1
SOLVER_AUTO, SOLVER_PREFACTORED, SOLVER_REGION, SOLVER_DENSE, SOLVER_NEWTON = 0, 1, 2, 3, 4
HOST, DEVICE = 0, 1
OPT_GRAPH, OPT_PLAN_LAYOUT, OPT_FUSED, OPT_COMPOSITE, OPT_MFMA, OPT_BRICK = 1, 2, 3, 4, 5, 6
ASM_QUADRATURE, ASM_QQF, ASM_PERTURBATION = 0, 1, 2

EXPORTS = [
    "ridg_workspace_bytes", "ridg_create", "ridg_set_state", "ridg_step", "ridg_get_state",
    "ridg_get_prediction", "ridg_get_info", "ridg_enable_timing", "ridg_get_timing", "ridg_set_option",
    "ridg_get_option", "ridg_autotune", "ridg_step_batch", "ridg_advance_static", "ridg_newton_stats", "ridg_assemble_jacobian", "ridg_synchronize",
    "ridg_destroy",
    "ridg_host_region_matrix", "ridg_host_prediction_operator", "ridg_host_spectral_radius",
    "ridg_error_string", "ridg_last_error",
]


class RidgProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("newton_max_iter", ctypes.c_int32),
        ("velocity", ctypes.c_double * 3),
        ("rot_center", ctypes.c_double * 2),
        ("vel_grad", ctypes.c_double * 9),
        ("length", ctypes.c_double * 3),
        ("precision", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class RidgInfo(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("theta", ctypes.c_int32),
        ("theta_t", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("n_elements", ctypes.c_int64),
        ("n_plans", ctypes.c_int64),
        ("n_tear_elements", ctypes.c_int64),
        ("n_dense_elements", ctypes.c_int64),
        ("n_taps", ctypes.c_int64),
        ("flops_predict", ctypes.c_double),
        ("flops_correct", ctypes.c_double),
        ("bytes_predict", ctypes.c_double),
        ("bytes_correct", ctypes.c_double),
        ("flops_composite", ctypes.c_double),
        ("bytes_composite", ctypes.c_double),
        ("basis", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("spectral_radius", ctypes.c_double),
        ("static_pivot_growth", ctypes.c_double),
    ]


class RidgTiming(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("predict_ms", ctypes.c_double),
        ("correct_ms", ctypes.c_double),
        ("max_step_ms", ctypes.c_double),
    ]


class RidgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libridg error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libridg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2101_01231_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER(RidgProblem)
        L.ridg_workspace_bytes.argtypes = [P, ctypes.POINTER(sz)]
        L.ridg_create.argtypes = [P, vp, sz, vp, ctypes.POINTER(vp)]
        L.ridg_set_state.argtypes = [vp, vp, sz, i32]
        L.ridg_step.argtypes = [vp, i32, dbl]
        L.ridg_get_state.argtypes = [vp, vp, sz, i32]
        L.ridg_get_prediction.argtypes = [vp, dbl, vp, sz, i32]
        L.ridg_get_info.argtypes = [vp, ctypes.POINTER(RidgInfo)]
        L.ridg_enable_timing.argtypes = [vp, i32]
        L.ridg_get_timing.argtypes = [vp, ctypes.POINTER(RidgTiming)]
        L.ridg_set_option.argtypes = [vp, i32, i64]
        L.ridg_get_option.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.ridg_autotune.argtypes = [vp, dbl, i32, ctypes.POINTER(dbl)]
        L.ridg_step_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(dbl), i32, vp]
        L.ridg_advance_static.argtypes = [P, vp, vp, sz, i32, dbl, vp]
        L.ridg_newton_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i64), i32]
        L.ridg_assemble_jacobian.argtypes = [i32, i32, i32, vp, i64, dbl, vp, vp]
        L.ridg_synchronize.argtypes = [vp]
        L.ridg_destroy.argtypes = [vp]
        L.ridg_host_region_matrix.argtypes = [P, i64, dbl, vp, sz]
        L.ridg_host_prediction_operator.argtypes = [P, dbl, vp, sz]
        L.ridg_host_spectral_radius.argtypes = [P, dbl, i32, ctypes.POINTER(dbl)]
        L.ridg_error_string.restype = ctypes.c_char_p
        L.ridg_error_string.argtypes = [ctypes.c_int]
        L.ridg_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("ridg_error_string", "ridg_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise RidgError(rc, lib().ridg_last_error().decode())
    return rc


def make_problem(dim, n, order, velocity=None, flux=FLUX_CONST, rot_center=(0.5, 0.5), vel_grad=None,
                 precision=FP64, refine_steps=0, solver=SOLVER_AUTO, basis=BASIS_P, length=None, newton_max_iter=0):
    p = RidgProblem()
    p.dim = dim
    n = tuple(n) if hasattr(n, "__len__") else (n,) * dim
    for i in range(3):
        p.n[i] = n[i] if i < len(n) else 1
    p.order = order
    p.basis = basis
    p.flux = flux
    p.newton_max_iter = newton_max_iter
    L = tuple(length or ())
    for i in range(3):
        p.length[i] = float(L[i]) if i < len(L) else 0.0
    v = tuple(velocity or ())
    for i in range(3):
        p.velocity[i] = float(v[i]) if i < len(v) else 0.0
    p.rot_center[0], p.rot_center[1] = rot_center
    if vel_grad is not None:
        for i, x in enumerate(np.asarray(vel_grad, dtype=np.float64).reshape(-1)):
            p.vel_grad[i] = x
    p.precision = precision
    p.refine_steps = refine_steps
    p.solver = solver
    p.reserved = 0
    return p


def assemble_jacobian(method, dim, order, w, dt_over_h, out=None, stream=None):
    """Volume Jacobian blocks of the Burgers flux on every element of w (a CUDA tensor
    [n_elements, theta_T], float64) by quadrature, QQF or perturbation (ridg_assemble_jacobian)."""
    import torch
    n, nt = w.shape
    if out is None:
        out = torch.empty((n, nt, nt), dtype=torch.float64, device=w.device)
    if stream is None:
        stream = torch.cuda.current_stream(w.device)
    _check(lib().ridg_assemble_jacobian(int(method), int(dim), int(order), ctypes.c_void_p(w.data_ptr()), int(n),
                                        float(dt_over_h), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream)))
    return out


def workspace_bytes(problem):
    out = ctypes.c_size_t()
    _check(lib().ridg_workspace_bytes(ctypes.byref(problem), ctypes.byref(out)))
    return out.value


def _sizes(problem):
    """(theta, theta_T) of the problem's basis family."""
    from math import comb
    d, M = problem.dim, problem.order
    if problem.basis == BASIS_Q:
        return M ** d, M ** (d + 1)
    return comb(M - 1 + d, d), comb(M + d, d + 1)


def host_region_matrix(problem, element, dt):
    d = problem.dim
    nt = _sizes(problem)[1]
    n = 3 ** d * nt
    A = np.empty((n, n))
    _check(lib().ridg_host_region_matrix(ctypes.byref(problem), element, dt, A.ctypes.data, A.size))
    return A


def host_prediction_operator(problem, dt):
    d = problem.dim
    ns, nt = _sizes(problem)
    G = np.empty((nt, 3 ** d * ns))
    _check(lib().ridg_host_prediction_operator(ctypes.byref(problem), dt, G.ctypes.data, G.size))
    return G


def host_spectral_radius(problem, dt, nk=64):
    """Von Neumann amplification of the constant-velocity step (host precompute, no device)."""
    out = ctypes.c_double()
    _check(lib().ridg_host_spectral_radius(ctypes.byref(problem), float(dt), int(nk), ctypes.byref(out)))
    return out.value


def advance_static(problem, q_in, q_out, n_steps, dt, stream=None):
    """ridg_advance_static on torch device tensors (state layout of set/get); no device allocation."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(q_in.device)
    return _check(lib().ridg_advance_static(ctypes.byref(problem), ctypes.c_void_p(q_in.data_ptr()),
                                            ctypes.c_void_p(q_out.data_ptr()), q_in.numel(), int(n_steps),
                                            float(dt), ctypes.c_void_p(stream.cuda_stream)))


def step_batch(sims, dts, n_steps, stream):
    """Advance several PREFACTORED simulations in shared launches on `stream` (a torch stream)."""
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in sims])
    d = (ctypes.c_double * n)(*[float(x) for x in dts])
    return _check(lib().ridg_step_batch(hs, n, d, int(n_steps), ctypes.c_void_p(stream.cuda_stream)))


class Simulation:
    """One RIDG problem resident on a GPU (workspace owned by a torch tensor)."""

    def __init__(self, problem, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.problem = problem
        self.device = torch.device(device)
        nbytes = workspace_bytes(problem)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().ridg_create(ctypes.byref(problem), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                 ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.info = RidgInfo()
        _check(lib().ridg_get_info(self.handle, ctypes.byref(self.info)))
        self.theta = self.info.theta
        self.theta_t = self.info.theta_t
        self.n_el = self.info.n_elements
        self.last_warning = RIDG_OK

    def get_info(self):
        """Sizes, cost model and the per-dt analyses of the handle (ridg_info)."""
        info = RidgInfo()
        _check(lib().ridg_get_info(self.handle, ctypes.byref(info)))
        return info

    def close(self):
        if getattr(self, "handle", None):
            lib().ridg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, q):
        torch = self.torch
        if isinstance(q, torch.Tensor) and q.is_cuda:
            q = q.contiguous().to(torch.float64)
            _check(lib().ridg_set_state(self.handle, ctypes.c_void_p(q.data_ptr()), q.numel(), DEVICE))
            self.synchronize()
        else:
            a = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
            _check(lib().ridg_set_state(self.handle, a.ctypes.data, a.size, HOST))

    def step(self, n_steps, dt):
        return _check(lib().ridg_step(self.handle, int(n_steps), float(dt)))

    def get_state(self, out=None):
        if out is not None:
            _check(lib().ridg_get_state(self.handle, ctypes.c_void_p(out.data_ptr()), out.numel(), DEVICE))
            return out
        a = np.empty((self.n_el, self.theta))
        self.last_warning = _check(lib().ridg_get_state(self.handle, a.ctypes.data, a.size, HOST))
        return a

    def newton_stats(self, reset=False):
        """Burgers: dict of the Newton counters since creation or the last reset (synchronises)."""
        mx, tot, sol, fail = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ridg_newton_stats(self.handle, ctypes.byref(mx), ctypes.byref(tot), ctypes.byref(sol),
                                       ctypes.byref(fail), 1 if reset else 0))
        return {"max_iters": mx.value, "total_iters": tot.value, "solves": sol.value, "failures": fail.value}

    def get_prediction(self, dt):
        a = np.empty((self.n_el, self.theta_t))
        _check(lib().ridg_get_prediction(self.handle, float(dt), a.ctypes.data, a.size, HOST))
        return a

    def enable_timing(self, on=True):
        _check(lib().ridg_enable_timing(self.handle, 1 if on else 0))

    def get_timing(self):
        t = RidgTiming()
        _check(lib().ridg_get_timing(self.handle, ctypes.byref(t)))
        return t

    def set_option(self, option, value):
        _check(lib().ridg_set_option(self.handle, int(option), int(value)))

    def get_option(self, option):
        v = ctypes.c_int64()
        _check(lib().ridg_get_option(self.handle, int(option), ctypes.byref(v)))
        return v.value

    def autotune(self, dt, steps=10):
        """Pick the fastest option set for this problem; returns ms per step (-1 if cached)."""
        out = ctypes.c_double()
        _check(lib().ridg_autotune(self.handle, float(dt), int(steps), ctypes.byref(out)))
        return out.value

    def synchronize(self):
        _check(lib().ridg_synchronize(self.handle))
