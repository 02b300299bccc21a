"""Python binding of libimexdg (MI355X / gfx950 IMEX-DG for the compressible Euler equations).

Argument marshalling only: every step of the method runs in the HIP kernels of libimexdg.so,
called through its C ABI (``include/imexdg.h``).  Device buffers are torch tensors on the ROCm
device; the HIP stream is torch's current stream.  The functions carry the names of the C entry
points; ``Solver`` bundles a context with its state.

The library must have been built (``python -m paper_2408_08129_amd.build`` or
``__graft_entry__.build()``); importing works without it, but every call raises if the shared
library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimexdg.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EDEVICE, DG_ENOCONV, DG_ENAN, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
DG_FP64, DG_FP32_INNER = 0, 1
DG_PREC_DIAGONAL, DG_PREC_CELL_FDM = 0, 1
ORO_FLAT, ORO_AGNESI, ORO_BELL, ORO_GAUSS_HILL, ORO_GAUSS_RIDGE = range(5)
ATM_ISOTHERMAL, ATM_STRATIFIED = range(2)
DG_IC_HYDROSTATIC_WIND = 0
MAX_RULES = 8

EXPORTED = ("dg_default_options", "dg_setup", "dg_footprint", "dg_mesh_info", "dg_set_stream", "dg_set_timing",
            "dg_sizes", "dg_cell_table", "dg_node_geometry", "dg_init_state",
            "dg_explicit_residual", "dg_implicit_term", "dg_apply_helmholtz", "dg_apply_preconditioner",
            "imex_rk2_step",
            "imex_rk2_step_batched", "dg_diagnostics", "dg_diagnostics_noalloc", "dg_last_error",
            "dg_destroy")


class dg_refine_rule(ctypes.Structure):
    _fields_ = [("zeta_max", ctypes.c_double), ("x_c", ctypes.c_double),
                ("half_width_x", ctypes.c_double), ("y_c", ctypes.c_double),
                ("half_width_y", ctypes.c_double)]


class dg_case_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nbase", ctypes.c_int32 * 3),
                ("length", ctypes.c_double * 3), ("periodic_x", ctypes.c_int32),
                ("periodic_y", ctypes.c_int32), ("n_rules", ctypes.c_int32),
                ("rules", dg_refine_rule * MAX_RULES), ("orography", ctypes.c_int32),
                ("oro", ctypes.c_double * 4), ("atmosphere", ctypes.c_int32),
                ("atm", ctypes.c_double * 3), ("sponge", ctypes.c_double * 5)]


class dg_options(ctypes.Structure):
    _fields_ = [("fp_iters", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
                ("gmres_maxit", ctypes.c_int32), ("gmres_rtol", ctypes.c_double),
                ("gmres_atol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("inner_restart", ctypes.c_int32),
                ("inner_maxit", ctypes.c_int32), ("penalty_beta", ctypes.c_double),
                ("preconditioner", ctypes.c_int32), ("quad_extra", ctypes.c_int32),
                ("enthalpy_split", ctypes.c_int32)]


class dg_step_stats(ctypes.Structure):
    _fields_ = [("gmres_iters", (ctypes.c_int32 * 8) * 2), ("outer_iters", (ctypes.c_int32 * 8) * 2),
                ("gmres_relres", (ctypes.c_double * 8) * 2), ("fp_incr", (ctypes.c_double * 8) * 2),
                ("t_phase_ms", ctypes.c_double * 8), ("t_kernel_ms", ctypes.c_double * 8),
                ("n_kernel", ctypes.c_int32 * 8), ("bytes_kernel", ctypes.c_double * 8),
                ("t_step_ms", ctypes.c_double),
                ("mass", ctypes.c_double), ("max_w", ctypes.c_double)]

    KERNEL_CLASSES = ("explicit_residual", "helmholtz_pass1", "helmholtz_pass2", "gs_dots",
                      "pointwise", "gs_update", "krylov_other", "operator_other")
    PHASES = ("explicit_residuals", "implicit_term", "stage_updates", "fixed_point_coefficients",
              "helmholtz_rhs", "krylov", "back_substitution", "checks_and_diagnostics")

    def as_dict(self, fp_iters: int = 8) -> dict:
        return {
            "gmres_iters": [[self.gmres_iters[s][l] for l in range(fp_iters)] for s in range(2)],
            "outer_iters": [[self.outer_iters[s][l] for l in range(fp_iters)] for s in range(2)],
            "gmres_relres": [[self.gmres_relres[s][l] for l in range(fp_iters)] for s in range(2)],
            "fp_incr": [[self.fp_incr[s][l] for l in range(fp_iters)] for s in range(2)],
            "t_phase_ms": {k: self.t_phase_ms[i] for i, k in enumerate(self.PHASES)},
            "t_kernel_ms": {k: self.t_kernel_ms[i] for i, k in enumerate(self.KERNEL_CLASSES)},
            "n_kernel": {k: self.n_kernel[i] for i, k in enumerate(self.KERNEL_CLASSES)},
            "bytes_kernel": {k: self.bytes_kernel[i] for i, k in enumerate(self.KERNEL_CLASSES)},
            "t_step_ms": self.t_step_ms, "mass": self.mass, "max_w": self.max_w,
        }


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("imexdg error %d: %s" % (status, msg))
        self.status = status


_lib = None


def _hip_runtimes() -> set:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def lib():
    """The loaded shared library; raises if it has not been built.

    torch ships its own HIP runtime under the same soname as the system one the library is linked
    against.  torch is imported first so that the library binds to torch's runtime; loading the
    library first would map two HIP/HSA runtimes into the process, which crashes at the first
    device call.  The load is checked for a single runtime."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libimexdg.so is not built (run paper_2408_08129_amd/build.py); "
                              "there is no CPU fallback")
        import torch  # noqa: F401  (binds the HIP runtime first)
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise ImportError("more than one HIP runtime is loaded in this process: %s" % sorted(rts))
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.dg_default_options.argtypes = [ctypes.POINTER(dg_options)]
        L.dg_default_options.restype = None
        L.dg_setup.argtypes = [ctypes.POINTER(dg_case_desc), i32, ctypes.POINTER(dg_options), vp,
                               ctypes.POINTER(vp)]
        L.dg_footprint.argtypes = [ctypes.POINTER(dg_case_desc), i32, ctypes.POINTER(dg_options),
                                   ctypes.POINTER(ctypes.c_size_t)]
        L.dg_mesh_info.argtypes = [ctypes.POINTER(dg_case_desc), i32, ctypes.POINTER(i64),
                                   ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.dg_set_stream.argtypes = [vp, vp]
        L.dg_set_timing.argtypes = [vp, i32]
        L.dg_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.dg_cell_table.argtypes = [vp, ctypes.POINTER(i32)]
        L.dg_node_geometry.argtypes = [vp, vp, vp, vp, vp]
        L.dg_init_state.argtypes = [vp, i32, ctypes.POINTER(d), ctypes.c_uint64, d, vp]
        L.dg_explicit_residual.argtypes = [vp, vp, vp]
        L.dg_implicit_term.argtypes = [vp, vp, vp]
        L.dg_apply_helmholtz.argtypes = [vp, d, vp, vp, vp, i32]
        L.dg_apply_preconditioner.argtypes = [vp, d, vp, vp, vp, i32]
        L.imex_rk2_step.argtypes = [vp, vp, d, ctypes.POINTER(dg_step_stats)]
        L.imex_rk2_step_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            ctypes.POINTER(d), i32, ctypes.POINTER(dg_step_stats),
                                            ctypes.POINTER(i32)]
        L.dg_diagnostics.argtypes = [vp, vp, ctypes.POINTER(d), ctypes.POINTER(d)]
        L.dg_diagnostics_noalloc.argtypes = [vp, vp, ctypes.POINTER(d), ctypes.POINTER(d)]
        L.dg_last_error.argtypes = [vp]
        L.dg_last_error.restype = ctypes.c_char_p
        L.dg_destroy.argtypes = [vp]
        L.dg_destroy.restype = None
        for name in EXPORTED:
            if name not in ("dg_default_options", "dg_last_error", "dg_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, ctx: int | None = None):
    if rc != DG_OK:
        raise DGError(rc, lib().dg_last_error(ctypes.c_void_p(ctx)).decode())


# ----------------------------------------------------------------------------------- descriptions
@dataclass
class Case:
    """Problem description (mirrors dg_case_desc)."""
    dim: int
    nbase: tuple
    length: tuple
    periodic: tuple = (1, 1)
    rules: list = field(default_factory=list)  # (zeta_max, x_c, half_width_x, y_c, half_width_y)
    orography: int = ORO_FLAT
    oro: tuple = (0.0, 1.0, 0.0, 0.0)
    atmosphere: int = ATM_ISOTHERMAL
    atm: tuple = (1.0e5, 250.0, 0.0)
    # absorbing layers: (top depth, top rate, lateral width, lateral rate, u_ref); rates 0 = off
    sponge: tuple = (0.0, 0.0, 0.0, 0.0, 0.0)

    def to_c(self) -> dg_case_desc:
        c = dg_case_desc()
        c.dim = self.dim
        for i in range(3):
            c.nbase[i] = int(self.nbase[i])
            c.length[i] = float(self.length[i])
        c.periodic_x, c.periodic_y = int(self.periodic[0]), int(self.periodic[1])
        if len(self.rules) > MAX_RULES:
            raise ValueError("too many refinement rules")
        c.n_rules = len(self.rules)
        for i, r in enumerate(self.rules):
            c.rules[i] = dg_refine_rule(*[float(v) for v in r])
        c.orography = self.orography
        for i in range(4):
            c.oro[i] = float(self.oro[i])
        c.atmosphere = self.atmosphere
        atm = list(self.atm) + [0.0] * (3 - len(self.atm))
        for i in range(3):
            c.atm[i] = float(atm[i])
        sp = list(self.sponge) + [0.0] * (5 - len(self.sponge))
        for i in range(5):
            c.sponge[i] = float(sp[i])
        return c


def options(**kw) -> dg_options:
    o = dg_options()
    lib().dg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ---------------------------------------------------------------------------- C-ABI-named calls
def dg_footprint(case: Case, degree: int, opt: dg_options | None = None) -> int:
    n = ctypes.c_size_t()
    cd = case.to_c()
    _check(lib().dg_footprint(ctypes.byref(cd), degree, ctypes.byref(opt) if opt else None, ctypes.byref(n)))
    return n.value


def dg_mesh_info(case: Case, degree: int, with_cells: bool = True):
    """(n_cells, n_hanging, cell table or None) -- host only, no device needed."""
    import numpy as np
    nc = ctypes.c_int64()
    nh = ctypes.c_int64()
    cd = case.to_c()
    _check(lib().dg_mesh_info(ctypes.byref(cd), degree, ctypes.byref(nc), ctypes.byref(nh), None))
    cells = None
    if with_cells:
        cells = np.zeros((nc.value, 4), dtype=np.int32)
        _check(lib().dg_mesh_info(ctypes.byref(cd), degree, ctypes.byref(nc), ctypes.byref(nh),
                                  cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return nc.value, nh.value, cells


def dg_setup(case: Case, degree: int, opt: dg_options | None = None, stream=None) -> int:
    h = ctypes.c_void_p()
    cd = case.to_c()
    _check(lib().dg_setup(ctypes.byref(cd), degree, ctypes.byref(opt) if opt else None,
                          ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
    return h.value


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def dg_init_state(ctx: int, U, ubar: float = 0.0, noise_seed: int = 0, noise_sigma_K: float = 0.0,
                  ic_kind: int = DG_IC_HYDROSTATIC_WIND):
    params = (ctypes.c_double * 4)(float(ubar), 0.0, 0.0, 0.0)
    _check(lib().dg_init_state(ctypes.c_void_p(ctx), ic_kind, params, ctypes.c_uint64(int(noise_seed)),
                               float(noise_sigma_K), _ptr(U)), ctx)


def dg_explicit_residual(ctx: int, U, R):
    _check(lib().dg_explicit_residual(ctypes.c_void_p(ctx), _ptr(U), _ptr(R)), ctx)


def dg_implicit_term(ctx: int, U, F):
    _check(lib().dg_implicit_term(ctypes.c_void_p(ctx), _ptr(U), _ptr(F)), ctx)


def dg_apply_helmholtz(ctx: int, dt_a: float, h, p, Ap, prec: int = DG_FP64):
    _check(lib().dg_apply_helmholtz(ctypes.c_void_p(ctx), float(dt_a), _ptr(h), _ptr(p), _ptr(Ap), prec), ctx)


def dg_apply_preconditioner(ctx: int, dt_a: float, h, v, z, prec: int = DG_FP64):
    _check(lib().dg_apply_preconditioner(ctypes.c_void_p(ctx), float(dt_a), _ptr(h), _ptr(v), _ptr(z), prec), ctx)


def imex_rk2_step(ctx: int, U, dt: float) -> dg_step_stats:
    st = dg_step_stats()
    _check(lib().imex_rk2_step(ctypes.c_void_p(ctx), _ptr(U), float(dt), ctypes.byref(st)), ctx)
    return st


def imex_rk2_step_batched(ctxs, Us, dts, raise_on_error: bool = True):
    """One step for every member; returns (stats list, status list)."""
    n = len(ctxs)
    C = (ctypes.c_void_p * n)(*ctxs)
    P = (ctypes.c_void_p * n)(*[u.data_ptr() for u in Us])
    T = (ctypes.c_double * n)(*[float(x) for x in dts])
    S = (dg_step_stats * n)()
    R = (ctypes.c_int32 * n)()
    rc = lib().imex_rk2_step_batched(C, P, T, n, S, R)
    if raise_on_error:
        _check(rc)
    return list(S), list(R)


def dg_diagnostics(ctx: int, U):
    m = ctypes.c_double()
    w = ctypes.c_double()
    _check(lib().dg_diagnostics(ctypes.c_void_p(ctx), _ptr(U), ctypes.byref(m), ctypes.byref(w)), ctx)
    return m.value, w.value


def dg_diagnostics_noalloc(ctx: int, U):
    m = ctypes.c_double()
    w = ctypes.c_double()
    _check(lib().dg_diagnostics_noalloc(ctypes.c_void_p(ctx), _ptr(U), ctypes.byref(m), ctypes.byref(w)), ctx)
    return m.value, w.value


def dg_destroy(ctx: int):
    lib().dg_destroy(ctypes.c_void_p(ctx))


class Solver:
    """A context plus convenience accessors; tensors are float64 on the current ROCm device."""

    def __init__(self, case: Case, degree: int, opt: dg_options | None = None, stream=None):
        import torch
        self.torch = torch
        self.case = case
        self.degree = degree
        self.opt = opt if opt is not None else options()
        self.stream = stream
        self.ctx = dg_setup(case, degree, self.opt, stream)
        nc = ctypes.c_int64()
        nn = ctypes.c_int64()
        nf = ctypes.c_int32()
        _check(lib().dg_sizes(ctypes.c_void_p(self.ctx), ctypes.byref(nc), ctypes.byref(nn), ctypes.byref(nf)))
        self.ncell, self.N, self.nf = nc.value, nn.value, nf.value
        self.dim = case.dim
        self.nloc = (degree + 1) ** case.dim

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                dg_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def close(self):
        self.__del__()

    def _sync(self):
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream()
        s.synchronize()

    def empty_state(self):
        return self.torch.empty((self.nf, self.N), dtype=self.torch.float64, device="cuda")

    def cell_table(self):
        import numpy as np
        out = np.zeros((self.ncell, 4), dtype=np.int32)
        _check(lib().dg_cell_table(ctypes.c_void_p(self.ctx), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def node_geometry(self):
        t = self.torch
        x, y, z, wJ = (t.empty(self.N, dtype=t.float64, device="cuda") for _ in range(4))
        _check(lib().dg_node_geometry(ctypes.c_void_p(self.ctx), _ptr(x), _ptr(y), _ptr(z), _ptr(wJ)))
        self._sync()
        return x, y, z, wJ

    def init_state(self, ubar: float = 0.0, noise_seed: int = 0, noise_sigma_K: float = 0.0):
        U = self.empty_state()
        dg_init_state(self.ctx, U, ubar, noise_seed, noise_sigma_K)
        return U

    def explicit_residual(self, U):
        R = self.torch.empty_like(U)
        dg_explicit_residual(self.ctx, U, R)
        return R

    def implicit_term(self, U):
        F = self.torch.empty_like(U)
        dg_implicit_term(self.ctx, U, F)
        return F

    def apply_helmholtz(self, dt_a, h, p, prec=DG_FP64):
        Ap = self.torch.empty_like(p)
        dg_apply_helmholtz(self.ctx, dt_a, h, p, Ap, prec)
        return Ap

    def apply_preconditioner(self, dt_a, h, v, prec=DG_FP64):
        z = self.torch.empty_like(v)
        dg_apply_preconditioner(self.ctx, dt_a, h, v, z, prec)
        return z

    def step(self, U, dt) -> dg_step_stats:
        return imex_rk2_step(self.ctx, U, dt)

    def diagnostics(self, U):
        return dg_diagnostics(self.ctx, U)

    def set_timing(self, on: bool = True):
        _check(lib().dg_set_timing(ctypes.c_void_p(self.ctx), 1 if on else 0))
