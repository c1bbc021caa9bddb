"""Python binding of librhmc (include/rhmc.h): argument marshalling only.

Every computation happens in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw device pointers and the caller's HIP
stream, and turns status codes into exceptions.  PyTorch only supplies device
memory and streams.  Importing works without a GPU; the first call into the
library raises if ``librhmc.so`` has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librhmc.so")

RHMC_OK = 0
RHMC_ERR_INVALID_ARG = -1
RHMC_ERR_NONFINITE = -2
RHMC_ERR_NOT_CONVERGED = -3
RHMC_ERR_HIP = -4
RHMC_ERR_OOM = -5
RHMC_ERR_UNSUPPORTED = -6

RHMC_PREC_FP64 = 0
RHMC_PREC_FP32 = 1
RHMC_LINKS_FP64_18 = 1
RHMC_LINKS_FP32_12 = 2
RHMC_LINKS_HILO_12 = 4
RHMC_LINKS_FP64_12 = 8
RHMC_LINKS_FP32_18 = 16
RHMC_MODE_FP64 = 0
RHMC_MODE_MIXED = 1

# every symbol the header declares, for the load check
EXPORTED = (
    "rhmc_solver_params_default", "rhmc_lattice_create", "rhmc_lattice_destroy",
    "rhmc_debug_neighbors", "rhmc_gauge_create", "rhmc_gauge_destroy", "rhmc_dslash_eo",
    "rhmc_apply_mdagm", "rhmc_apply_mdagm_static", "rhmc_multishift_cg", "rhmc_rational_apply",
    "rhmc_tune_dslash",
    "rhmc_dslash_variant", "rhmc_set_dslash_variant", "rhmc_pf_phi", "rhmc_pf_action",
    "rhmc_pf_force", "rhmc_gauge_action", "rhmc_gauge_force_kick", "rhmc_pf_force_kick",
    "rhmc_update_links", "rhmc_kinetic", "rhmc_gauge_links", "rhmc_md_params_default",
    "rhmc_md_integrate", "rhmc_trajectory",
    "rhmc_status_string", "rhmc_last_error",
)


class RhmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rhmc status {status}: {message}")
        self.status = status


class rhmc_solver_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("mode", C.c_int32),
                ("reliable_every", C.c_int32), ("refine", C.c_int32), ("block", C.c_int32),
                ("use_graph", C.c_int32), ("poll_every", C.c_int32), ("tune", C.c_int32),
                ("per_shift", C.c_int32), ("fp64_head", C.c_double), ("two_pass", C.c_int32)]


class rhmc_solver_stats(C.Structure):
    _fields_ = [("iterations", C.POINTER(C.c_int32)), ("true_residual", C.POINTER(C.c_double)),
                ("refine_iterations", C.POINTER(C.c_int32)), ("total_iterations", C.c_int32),
                ("reliable_updates", C.c_int32), ("refine_rounds", C.c_int32),
                ("time_ms", C.c_double), ("max_true_residual", C.c_double),
                ("fp64_head_iterations", C.c_int32), ("head_ms", C.c_double),
                ("krylov_ms", C.c_double), ("check_ms", C.c_double), ("refine_ms", C.c_double)]


class rhmc_rational(C.Structure):
    _fields_ = [("alpha0", C.c_double), ("npole", C.c_int32),
                ("alpha", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double))]


class rhmc_md_params(C.Structure):
    _fields_ = [("beta", C.c_double), ("mass", C.c_double), ("tau", C.c_double),
                ("n_md", C.c_int32), ("gauge_steps", C.c_int32), ("lambda_", C.c_double),
                ("force_rational", C.POINTER(rhmc_rational)), ("solver", rhmc_solver_params)]


class rhmc_md_stats(C.Structure):
    _fields_ = [("fermion_forces", C.c_int32), ("gauge_forces", C.c_int32),
                ("link_updates", C.c_int32), ("cg_iterations", C.c_int64),
                ("max_true_residual", C.c_double), ("time_ms", C.c_double)]


class rhmc_hmc_params(C.Structure):
    _fields_ = [("md", rhmc_md_params), ("heatbath_rational", C.POINTER(rhmc_rational)),
                ("action_rational", C.POINTER(rhmc_rational)),
                ("metropolis_solver", rhmc_solver_params)]


class rhmc_trajectory_stats(C.Structure):
    _fields_ = [("kinetic", C.c_double * 2), ("gauge_action", C.c_double * 2),
                ("pf_action", C.c_double * 2), ("dH", C.c_double), ("accepted", C.c_int32),
                ("md", rhmc_md_stats), ("time_ms", C.c_double)]


_lib = None


def load():
    """Load librhmc.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, u32, f64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_double
    sig = {
        "rhmc_solver_params_default": (None, [C.POINTER(rhmc_solver_params)]),
        "rhmc_lattice_create": (i32, [C.POINTER(C.c_int32), i32, C.POINTER(vp)]),
        "rhmc_lattice_destroy": (None, [vp]),
        "rhmc_debug_neighbors": (i32, [vp, i32, vp, vp]),
        "rhmc_gauge_create": (i32, [vp, vp, u32, vp, C.POINTER(vp)]),
        "rhmc_gauge_destroy": (None, [vp]),
        "rhmc_dslash_eo": (i32, [vp, i32, i32, i32, vp, vp, vp]),
        "rhmc_apply_mdagm": (i32, [vp, f64, i32, i32, vp, vp, vp]),
        "rhmc_apply_mdagm_static": (i32, [vp, f64, i32, i32, vp, vp, vp]),
        "rhmc_multishift_cg": (i32, [vp, f64, i32, C.POINTER(C.c_double), i32, vp, vp,
                                     C.POINTER(rhmc_solver_params), C.POINTER(rhmc_solver_stats), vp]),
        "rhmc_rational_apply": (i32, [vp, f64, C.POINTER(rhmc_rational), i32, vp, vp,
                                      C.POINTER(rhmc_solver_params), C.POINTER(rhmc_solver_stats), vp]),
        "rhmc_tune_dslash": (i32, [vp, i32, i32, vp, vp, vp]),
        "rhmc_pf_force": (i32, [vp, f64, C.POINTER(rhmc_rational), i32, vp, vp,
                                C.POINTER(rhmc_solver_params), C.POINTER(rhmc_solver_stats), vp]),
        "rhmc_pf_phi": (i32, [vp, f64, i32, vp, vp, vp, vp]),
        "rhmc_pf_action": (i32, [vp, f64, C.POINTER(rhmc_rational), i32, vp, C.POINTER(C.c_double),
                                 C.POINTER(rhmc_solver_params), C.POINTER(rhmc_solver_stats), vp]),
        "rhmc_dslash_variant": (i32, [vp, i32, i32, C.POINTER(C.c_int32)]),
        "rhmc_set_dslash_variant": (i32, [vp, i32, i32, i32]),
        "rhmc_gauge_action": (i32, [vp, f64, C.POINTER(C.c_double), vp]),
        "rhmc_gauge_force_kick": (i32, [vp, f64, f64, vp, vp]),
        "rhmc_pf_force_kick": (i32, [vp, f64, C.POINTER(rhmc_rational), i32, vp, f64, vp,
                                     C.POINTER(rhmc_solver_params), C.POINTER(rhmc_solver_stats), vp]),
        "rhmc_update_links": (i32, [vp, f64, vp, vp]),
        "rhmc_kinetic": (i32, [vp, vp, C.POINTER(C.c_double), vp]),
        "rhmc_gauge_links": (i32, [vp, vp, vp]),
        "rhmc_md_params_default": (None, [C.POINTER(rhmc_md_params)]),
        "rhmc_md_integrate": (i32, [vp, C.POINTER(rhmc_md_params), i32, vp, vp,
                                    C.POINTER(rhmc_md_stats), vp]),
        "rhmc_trajectory": (i32, [vp, C.POINTER(rhmc_hmc_params), i32, vp, vp, f64,
                                  C.POINTER(rhmc_trajectory_stats), vp]),
        "rhmc_status_string": (C.c_char_p, [i32]),
        "rhmc_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != RHMC_OK:
        lib = load()
        raise RhmcError(status, lib.rhmc_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class Lattice:
    """Owns an rhmc_lattice handle."""

    def __init__(self, handle, L, t_bc):
        self.handle = handle
        self.L = tuple(int(x) for x in L)
        self.t_bc = t_bc
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.Vh = self.V // 2

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rhmc_lattice_destroy(self.handle)
            self.handle = None


class Gauge:
    """Owns an rhmc_gauge handle (packed links + solver workspace on the device)."""

    def __init__(self, handle, lattice: Lattice):
        self.handle = handle
        self.lattice = lattice

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rhmc_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def rhmc_solver_params_default() -> rhmc_solver_params:
    p = rhmc_solver_params()
    load().rhmc_solver_params_default(C.byref(p))
    return p


def solver_params(**kw) -> rhmc_solver_params:
    p = rhmc_solver_params_default()
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def rhmc_lattice_create(L, t_bc: int = -1) -> Lattice:
    lib = load()
    arr = (C.c_int32 * 4)(*[int(x) for x in L])
    h = C.c_void_p()
    _check(lib.rhmc_lattice_create(arr, int(t_bc), C.byref(h)))
    return Lattice(h, L, t_bc)


def rhmc_debug_neighbors(lat: Lattice, parity: int):
    lib = load()
    nb = np.zeros((lat.Vh, 8), dtype=np.int32)
    sg = np.zeros((lat.Vh, 8), dtype=np.int32)
    _check(lib.rhmc_debug_neighbors(lat.handle, int(parity), nb.ctypes.data_as(C.c_void_p),
                                    sg.ctypes.data_as(C.c_void_p)))
    return nb, sg


def rhmc_gauge_create(lat: Lattice, links: np.ndarray, flags: int = 0, stream=None) -> Gauge:
    lib = load()
    Lx, Ly, Lz, Lt = lat.L
    links = np.ascontiguousarray(links, dtype=np.complex128)
    if links.shape != (Lt, Lz, Ly, Lx, 4, 3, 3):
        raise ValueError(f"links must have shape {(Lt, Lz, Ly, Lx, 4, 3, 3)}, got {links.shape}")
    h = C.c_void_p()
    _check(lib.rhmc_gauge_create(lat.handle, links.ctypes.data_as(C.c_void_p), int(flags),
                                 _stream(stream), C.byref(h)))
    return Gauge(h, lat)


def _vec_dtype(prec):
    import torch

    return torch.complex128 if prec == RHMC_PREC_FP64 else torch.complex64


def vec_shape(prec: int, nrhs: int, Vh: int):
    """Tensor shape of a vector set at the ABI: complex128 [nrhs][3][Vh]; complex64
    [3][Vh] for one vector and [ceil(nrhs/2)][3][Vh][2] (pairs) for two or more."""
    if prec == RHMC_PREC_FP32 and nrhs >= 2:
        return ((nrhs + 1) // 2, 3, Vh, 2)
    return (nrhs, 3, Vh)


def rhmc_dslash_eo(g: Gauge, out_parity: int, prec: int, nrhs: int, inp, out, stream=None):
    shape = vec_shape(prec, nrhs, g.lattice.Vh)
    dt = _vec_dtype(prec)
    _check(load().rhmc_dslash_eo(g.handle, int(out_parity), int(prec), int(nrhs),
                                 _ptr(inp, dt, shape, "in"), _ptr(out, dt, shape, "out"),
                                 _stream(stream)))


def rhmc_apply_mdagm(g: Gauge, m: float, prec: int, nrhs: int, inp, out, stream=None):
    shape = vec_shape(prec, nrhs, g.lattice.Vh)
    dt = _vec_dtype(prec)
    _check(load().rhmc_apply_mdagm(g.handle, float(m), int(prec), int(nrhs),
                                   _ptr(inp, dt, shape, "in"), _ptr(out, dt, shape, "out"),
                                   _stream(stream)))


def rhmc_apply_mdagm_static(g: Gauge, m: float, prec: int, nrhs: int, inp, out, stream=None):
    """rhmc_apply_mdagm with its temporaries in the library's static device
    scratch (no allocation)."""
    shape = vec_shape(prec, nrhs, g.lattice.Vh)
    dt = _vec_dtype(prec)
    _check(load().rhmc_apply_mdagm_static(g.handle, float(m), int(prec), int(nrhs),
                                          _ptr(inp, dt, shape, "in"),
                                          _ptr(out, dt, shape, "out"), _stream(stream)))


class _Stats:
    def __init__(self, nrhs, nshift):
        self.iterations = np.zeros(nrhs * nshift, dtype=np.int32)
        self.true_residual = np.zeros(nrhs * nshift, dtype=np.float64)
        self.refine_iterations = np.zeros(nrhs * nshift, dtype=np.int32)
        self.c = rhmc_solver_stats()
        self.c.iterations = self.iterations.ctypes.data_as(C.POINTER(C.c_int32))
        self.c.true_residual = self.true_residual.ctypes.data_as(C.POINTER(C.c_double))
        self.c.refine_iterations = self.refine_iterations.ctypes.data_as(C.POINTER(C.c_int32))

    def as_dict(self, nrhs, nshift, status):
        return dict(
            status=status,
            iterations=self.iterations.reshape(nrhs, nshift).copy(),
            true_residual=self.true_residual.reshape(nrhs, nshift).copy(),
            refine_iterations=self.refine_iterations.reshape(nrhs, nshift).copy(),
            total_iterations=int(self.c.total_iterations),
            reliable_updates=int(self.c.reliable_updates),
            refine_rounds=int(self.c.refine_rounds),
            time_ms=float(self.c.time_ms),
            max_true_residual=float(self.c.max_true_residual),
            fp64_head_iterations=int(self.c.fp64_head_iterations),
            head_ms=float(self.c.head_ms),
            krylov_ms=float(self.c.krylov_ms),
            check_ms=float(self.c.check_ms),
            refine_ms=float(self.c.refine_ms),
        )


def rhmc_multishift_cg(g: Gauge, m: float, shifts, b, x, params=None, stream=None,
                       allow_not_converged=False):
    """x[r, i] = (A + shifts[i])^-1 b[r]; returns the solver statistics."""
    import torch

    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    nshift = shifts.size
    nrhs = int(b.shape[0])
    Vh = g.lattice.Vh
    pb = _ptr(b, torch.complex128, (nrhs, 3, Vh), "b")
    px = _ptr(x, torch.complex128, (nrhs, nshift, 3, Vh), "x")
    st = _Stats(nrhs, nshift)
    prm = params if params is not None else rhmc_solver_params_default()
    status = load().rhmc_multishift_cg(g.handle, float(m), nshift,
                                       shifts.ctypes.data_as(C.POINTER(C.c_double)), nrhs, pb, px,
                                       C.byref(prm), C.byref(st.c), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return st.as_dict(nrhs, nshift, status)


def rhmc_rational_apply(g: Gauge, m: float, alpha0: float, alpha, beta, b, y, params=None,
                        stream=None, allow_not_converged=False):
    """y[r] = alpha0 b[r] + sum_i alpha_i (A + beta_i)^-1 b[r]; returns statistics."""
    import torch

    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    if alpha.shape != beta.shape or alpha.ndim != 1:
        raise ValueError("alpha and beta must be 1-D of equal length")
    nrhs = int(b.shape[0])
    Vh = g.lattice.Vh
    pb = _ptr(b, torch.complex128, (nrhs, 3, Vh), "b")
    py = _ptr(y, torch.complex128, (nrhs, 3, Vh), "y")
    rat = rhmc_rational(float(alpha0), alpha.size, alpha.ctypes.data_as(C.POINTER(C.c_double)),
                        beta.ctypes.data_as(C.POINTER(C.c_double)))
    st = _Stats(nrhs, alpha.size)
    prm = params if params is not None else rhmc_solver_params_default()
    status = load().rhmc_rational_apply(g.handle, float(m), C.byref(rat), nrhs, pb, py,
                                        C.byref(prm), C.byref(st.c), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return st.as_dict(nrhs, alpha.size, status)


def rhmc_pf_phi(g: Gauge, m: float, r_even, r_odd, phi, stream=None):
    """phi_e = m R_e - D_eo R_o (Phi-algorithm pseudofermion field, FP64)."""
    import torch

    nrhs = int(r_even.shape[0])
    Vh = g.lattice.Vh
    shape = (nrhs, 3, Vh)
    _check(load().rhmc_pf_phi(g.handle, float(m), nrhs, _ptr(r_even, torch.complex128, shape, "r_even"),
                              _ptr(r_odd, torch.complex128, shape, "r_odd"),
                              _ptr(phi, torch.complex128, shape, "phi"), _stream(stream)))


def rhmc_pf_action(g: Gauge, m: float, alpha0: float, alpha, beta, phi, params=None, stream=None,
                   allow_not_converged=False):
    """S[r] = Re <phi_r, r(A) phi_r>; returns (S as numpy float64[nrhs], statistics)."""
    import torch

    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    if alpha.shape != beta.shape or alpha.ndim != 1:
        raise ValueError("alpha and beta must be 1-D of equal length")
    nrhs = int(phi.shape[0])
    Vh = g.lattice.Vh
    pp = _ptr(phi, torch.complex128, (nrhs, 3, Vh), "phi")
    rat = rhmc_rational(float(alpha0), alpha.size, alpha.ctypes.data_as(C.POINTER(C.c_double)),
                        beta.ctypes.data_as(C.POINTER(C.c_double)))
    S = np.zeros(nrhs, dtype=np.float64)
    st = _Stats(nrhs, alpha.size)
    prm = params if params is not None else rhmc_solver_params_default()
    status = load().rhmc_pf_action(g.handle, float(m), C.byref(rat), nrhs, pp,
                                   S.ctypes.data_as(C.POINTER(C.c_double)), C.byref(prm),
                                   C.byref(st.c), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return S, st.as_dict(nrhs, alpha.size, status)


def rhmc_pf_force(g: Gauge, m: float, alpha0: float, alpha, beta, phi, force, params=None,
                  stream=None, allow_not_converged=False):
    """force = TA(U M) of S = sum_r phi_r^dagger r(A) phi_r; returns statistics."""
    import torch

    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    if alpha.shape != beta.shape or alpha.ndim != 1:
        raise ValueError("alpha and beta must be 1-D of equal length")
    nrhs = int(phi.shape[0])
    Lx, Ly, Lz, Lt = g.lattice.L
    pp = _ptr(phi, torch.complex128, (nrhs, 3, g.lattice.Vh), "phi")
    pf = _ptr(force, torch.complex128, (Lt, Lz, Ly, Lx, 4, 3, 3), "force")
    rat = rhmc_rational(float(alpha0), alpha.size, alpha.ctypes.data_as(C.POINTER(C.c_double)),
                        beta.ctypes.data_as(C.POINTER(C.c_double)))
    st = _Stats(nrhs, alpha.size)
    prm = params if params is not None else rhmc_solver_params_default()
    status = load().rhmc_pf_force(g.handle, float(m), C.byref(rat), nrhs, pp, pf, C.byref(prm),
                                  C.byref(st.c), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return st.as_dict(nrhs, alpha.size, status)


def rhmc_tune_dslash(g: Gauge, prec: int, nrhs: int, inp, out, stream=None):
    """Time every launch variant of the hopping kernel and keep the fastest."""
    shape = vec_shape(prec, nrhs, g.lattice.Vh)
    dt = _vec_dtype(prec)
    _check(load().rhmc_tune_dslash(g.handle, int(prec), int(nrhs), _ptr(inp, dt, shape, "in"),
                                   _ptr(out, dt, shape, "out"), _stream(stream)))


def rhmc_dslash_variant(g: Gauge, prec: int, nrhs: int) -> int:
    """Launch variant of the hopping kernel in use for (prec, nrhs)."""
    v = C.c_int32(-1)
    _check(load().rhmc_dslash_variant(g.handle, int(prec), int(nrhs), C.byref(v)))
    return v.value


def rhmc_set_dslash_variant(g: Gauge, prec: int, nrhs: int, variant: int):
    """Pin the hopping kernel's launch variant for (prec, nrhs)."""
    _check(load().rhmc_set_dslash_variant(g.handle, int(prec), int(nrhs), int(variant)))


# ------------------------------------------------------------------ molecular dynamics
class Rational:
    """An rhmc_rational together with the host arrays it points into."""

    def __init__(self, alpha0, alpha, beta):
        self.alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        if self.alpha.shape != self.beta.shape or self.alpha.ndim != 1:
            raise ValueError("alpha and beta must be 1-D of equal length")
        self.c = rhmc_rational(float(alpha0), self.alpha.size,
                               self.alpha.ctypes.data_as(C.POINTER(C.c_double)),
                               self.beta.ctypes.data_as(C.POINTER(C.c_double)))

    @classmethod
    def of(cls, r):
        """From any object with alpha0, alpha, beta attributes."""
        return r if isinstance(r, cls) else cls(r.alpha0, r.alpha, r.beta)


def _mom_shape(g: Gauge):
    return (8, 4, 2, g.lattice.Vh)


def rhmc_gauge_action(g: Gauge, beta: float, stream=None) -> float:
    S = C.c_double()
    _check(load().rhmc_gauge_action(g.handle, float(beta), C.byref(S), _stream(stream)))
    return S.value


def rhmc_gauge_force_kick(g: Gauge, beta: float, eps: float, mom, stream=None):
    """mom -= eps * (algebra coefficients of the plaquette-action force)."""
    import torch

    _check(load().rhmc_gauge_force_kick(g.handle, float(beta), float(eps),
                                        _ptr(mom, torch.float64, _mom_shape(g), "mom"),
                                        _stream(stream)))


def rhmc_pf_force_kick(g: Gauge, m: float, rational, phi, eps: float, mom, params=None,
                       stream=None, allow_not_converged=False):
    """mom -= eps * (algebra coefficients of the pseudofermion force); returns statistics."""
    import torch

    rat = Rational.of(rational)
    npf = int(phi.shape[0])
    pp = _ptr(phi, torch.complex128, (npf, 3, g.lattice.Vh), "phi")
    pm = _ptr(mom, torch.float64, _mom_shape(g), "mom")
    st = _Stats(npf, rat.alpha.size)
    prm = params if params is not None else rhmc_solver_params_default()
    status = load().rhmc_pf_force_kick(g.handle, float(m), C.byref(rat.c), npf, pp, float(eps), pm,
                                       C.byref(prm), C.byref(st.c), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return st.as_dict(npf, rat.alpha.size, status)


def rhmc_update_links(g: Gauge, eps: float, mom, stream=None):
    """U -> reunitarised exp(i eps H) U in every link storage of g."""
    import torch

    _check(load().rhmc_update_links(g.handle, float(eps),
                                    _ptr(mom, torch.float64, _mom_shape(g), "mom"), _stream(stream)))


def rhmc_kinetic(g: Gauge, mom, stream=None) -> float:
    import torch

    K = C.c_double()
    _check(load().rhmc_kinetic(g.handle, _ptr(mom, torch.float64, _mom_shape(g), "mom"),
                               C.byref(K), _stream(stream)))
    return K.value


def rhmc_gauge_links(g: Gauge, out, stream=None):
    """out (device complex128 [Lt][Lz][Ly][Lx][4][3][3]) = the current FP64 links."""
    import torch

    Lx, Ly, Lz, Lt = g.lattice.L
    _check(load().rhmc_gauge_links(g.handle, _ptr(out, torch.complex128, (Lt, Lz, Ly, Lx, 4, 3, 3),
                                                  "links"), _stream(stream)))


class MDParams:
    """rhmc_md_params with its rational kept alive; keyword names as in the C
    struct (lambda_ for lambda), force_rational any object with alpha0, alpha,
    beta, solver an rhmc_solver_params."""

    def __init__(self, force_rational, **kw):
        self.c = rhmc_md_params()
        load().rhmc_md_params_default(C.byref(self.c))
        self.rational = Rational.of(force_rational)
        self.c.force_rational = C.pointer(self.rational.c)
        for k, v in kw.items():
            if k == "lambda":
                k = "lambda_"
            if not hasattr(self.c, k):
                raise KeyError(k)
            setattr(self.c, k, v)


def _md_stats_dict(s: rhmc_md_stats):
    return dict(fermion_forces=s.fermion_forces, gauge_forces=s.gauge_forces,
                link_updates=s.link_updates, cg_iterations=int(s.cg_iterations),
                max_true_residual=s.max_true_residual, time_ms=s.time_ms)


def rhmc_md_integrate(g: Gauge, params: MDParams, phi, mom, stream=None,
                      allow_not_converged=False):
    """Multi-step 2MN molecular dynamics over params.tau; links and mom in place."""
    import torch

    npf = int(phi.shape[0])
    pp = _ptr(phi, torch.complex128, (npf, 3, g.lattice.Vh), "phi")
    pm = _ptr(mom, torch.float64, _mom_shape(g), "mom")
    st = rhmc_md_stats()
    status = load().rhmc_md_integrate(g.handle, C.byref(params.c), npf, pp, pm, C.byref(st),
                                      _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    d = _md_stats_dict(st)
    d["status"] = status
    return d


class HMCParams:
    """rhmc_hmc_params: MD parameters, the heat-bath and action rationals and
    the solver parameters of the Metropolis solves."""

    def __init__(self, md: MDParams, heatbath_rational, action_rational, metropolis_solver=None):
        self.md = md
        self.hb = Rational.of(heatbath_rational)
        self.act = Rational.of(action_rational)
        self.c = rhmc_hmc_params()
        self.c.md = md.c
        self.c.heatbath_rational = C.pointer(self.hb.c)
        self.c.action_rational = C.pointer(self.act.c)
        self.c.metropolis_solver = (metropolis_solver if metropolis_solver is not None
                                    else rhmc_solver_params_default())


def rhmc_trajectory(g: Gauge, params: HMCParams, R, mom, u: float, stream=None,
                    allow_not_converged=False):
    """One trajectory (heat bath, MD, Metropolis); returns its statistics."""
    import torch

    npf = int(R.shape[0])
    pr = _ptr(R, torch.complex128, (npf, 3, g.lattice.Vh), "R")
    pm = _ptr(mom, torch.float64, _mom_shape(g), "mom")
    st = rhmc_trajectory_stats()
    status = load().rhmc_trajectory(g.handle, C.byref(params.c), npf, pr, pm, float(u),
                                    C.byref(st), _stream(stream))
    if not (allow_not_converged and status == RHMC_ERR_NOT_CONVERGED):
        _check(status)
    return dict(status=status, kinetic=tuple(st.kinetic), gauge_action=tuple(st.gauge_action),
                pf_action=tuple(st.pf_action), dH=st.dH, accepted=bool(st.accepted),
                md=_md_stats_dict(st.md), time_ms=st.time_ms)


def rhmc_status_string(status: int) -> str:
    return load().rhmc_status_string(int(status)).decode()


def rhmc_last_error() -> str:
    return load().rhmc_last_error().decode()
