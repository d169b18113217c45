"""Python binding of the MI355X FLD radiation-energy step library (``libfld.so``).

Argument marshalling only: every computation runs in the HIP kernels behind
the C ABI of ``include/fld.h``.  PyTorch provides device memory (the plan
workspace and the fields are torch tensors) and streams.  The module-level
functions carry the C names; :class:`Plan` is a small convenience wrapper.

Importing this module loads the in-tree ``libfld.so`` and raises if it is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfld.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2104_03968_amd/build.py` "
        "(hipcc, gfx950). There is no CPU fallback.")
# Device memory and streams come from torch, so the library must run on the same HIP
# runtime as torch.  torch puts its runtime in the process's global symbol scope;
# importing it before the library is loaded makes every HIP symbol of libfld.so --
# including the kernel registration done while it loads -- bind to that runtime
# instead of a second copy.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# ---- constants (include/fld.h) ---------------------------------------------------------
FLD_OK = 0
FLD_PENDING = 1
FLD_ERR_INVALID_ARG = -1
FLD_ERR_BAD_INPUT = -2
FLD_ERR_NOT_CONVERGED = -3
FLD_ERR_TOO_LARGE = -4
FLD_ERR_UNKNOWN_TICKET = -5
FLD_ERR_HIP = -6
FLD_ERR_NO_WORKSPACE = -7
FLD_ERR_UNSUPPORTED = -8
FLD_ERR_SHUTDOWN = -9
FLD_LIMITER_LP = 0
FLD_LIMITER_DIFFUSION = 1
FLD_LIMITER_MINERBO = 2
FLD_LIMITER_LP_EXACT = 3
LIMITER_CODES = {"lp": FLD_LIMITER_LP, "diffusion": FLD_LIMITER_DIFFUSION, "minerbo": FLD_LIMITER_MINERBO,
                 "lp_exact": FLD_LIMITER_LP_EXACT}
FLD_IMEX_EULER = 0
FLD_IMEX_MIDPOINT = 1
IMEX_SCHEMES = {"euler": FLD_IMEX_EULER, "midpoint": FLD_IMEX_MIDPOINT}
FLD_BC_ZERO_FLUX = 0
FLD_BC_FIXED_GRADIENT = 1
FLD_BC_DIRICHLET = 2
FLD_BC_PERIODIC = 3
FLD_BC_CONTINUOUS = 4
FLD_PREC_FP64 = 0
FLD_PREC_MIXED = 1
FLD_COARSE_REDISCRETISED = 0
FLD_COARSE_GALERKIN = 1
COARSE_OPS = {"rediscretised": FLD_COARSE_REDISCRETISED, "galerkin": FLD_COARSE_GALERKIN}
FLD_KERNEL_SMOOTH = 0
FLD_KERNEL_RESIDUAL = 1
FLD_KERNEL_RESTRICT = 2
FLD_KERNEL_PROLONG = 3
FLD_KERNEL_COEFF = 4
FLD_KERNEL_VCYCLE = 5
FLD_KERNEL_EXCHANGE = 6
FLD_KERNEL_DOWN = 7
FLD_KERNEL_UP = 8
FLD_KERNEL_TAIL = 9
FLD_KERNEL_SWEEP3 = 10
FLD_KERNEL_MG = 11
FLD_CYCLE_ITERATION = 0
FLD_CYCLE_MG = 1
FLD_CYCLE_FMG = 2


class fld_grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3)]


class fld_opts(C.Structure):
    _fields_ = [("c", C.c_double), ("limiter", C.c_int32), ("bc", C.c_int32 * 6),
                ("precision", C.c_int32), ("rtol", C.c_double), ("max_cycles", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("use_graph", C.c_int32),
                ("autotune", C.c_int32), ("krylov", C.c_int32), ("fused", C.c_int32),
                ("tile_rows", C.c_int32), ("tile_wide", C.c_int32), ("max_blocks", C.c_int32),
                ("tile_depth", C.c_int32), ("fused3_levels", C.c_int32), ("bc_grad", C.c_double * 6),
                ("tile_rows_coarse", C.c_int32), ("fmg", C.c_int32), ("coarse_op", C.c_int32),
                ("fmg_depths", C.c_int32), ("bc_value", C.c_double * 6), ("tile_rows_up", C.c_int32),
                ("nu_coarse", C.c_int32)]


class fld_tuning(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("tile_wide", C.c_int32), ("max_blocks", C.c_int32),
                ("source", C.c_int32), ("candidates", C.c_int32), ("vcycle_us", C.c_double),
                ("tile_depth", C.c_int32), ("fused3", C.c_int32), ("fused3_levels", C.c_int32),
                ("tile_rows_coarse", C.c_int32), ("tile_rows_up", C.c_int32), ("march_levels", C.c_int32),
                ("march_rows", C.c_int32), ("pq_rows", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fld_moments_out(C.Structure):
    _fields_ = [("F", C.c_void_p * 3), ("f_r", C.c_void_p * 3), ("edd", C.c_void_p), ("P", C.c_void_p * 6),
                ("tiring", C.c_void_p), ("E_out", C.c_void_p)]


class fld_stats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32), ("rel_residual", C.c_double),
                ("q_b", C.c_double), ("b_norm", C.c_double), ("b_sum", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fld_gas(C.Structure):
    _fields_ = [("c", C.c_double), ("a_rad", C.c_double), ("c_v", C.c_double),
                ("max_halley", C.c_int32), ("root_rtol", C.c_double)]


class fld_level_view(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("x", C.c_void_p), ("b", C.c_void_p),
                ("w", C.c_void_p * 3), ("x32", C.c_void_p), ("b32", C.c_void_p),
                ("w32", C.c_void_p * 3), ("ad", C.c_void_p)]


class fld_server_opts(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("precision", C.c_int32), ("rtol", C.c_double),
                ("max_cycles", C.c_int32), ("c", C.c_double), ("limiter", C.c_int32),
                ("cycles_per_round", C.c_int32)]


class fld_request(C.Structure):
    _fields_ = [("grid", fld_grid), ("dt", C.c_double), ("E_in", C.c_void_p), ("kappa_rho", C.c_void_p),
                ("inputs_on_device", C.c_int32), ("stream", C.c_void_p)]


class fld_result(C.Structure):
    _fields_ = [("E_out", C.c_void_p), ("stats", fld_stats), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


class fld_server_info(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("rounds", C.c_int64), ("cells_done", C.c_int64),
                ("pending", C.c_int32), ("resident", C.c_int32), ("arena_bytes", C.c_size_t),
                ("arena_free", C.c_size_t), ("error", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)
_sig = {
    "fld_version": (C.c_int32, []),
    "fld_strerror": (C.c_char_p, [C.c_int32]),
    "fld_last_error": (C.c_char_p, []),
    "fld_opts_default": (None, [C.POINTER(fld_opts)]),
    "fld_gas_default": (None, [C.POINTER(fld_gas)]),
    "fld_plan_create": (C.c_int32, [C.POINTER(fld_grid), C.c_int32, C.POINTER(fld_opts), _PP]),
    "fld_plan_destroy": (C.c_int32, [_P]),
    "fld_plan_workspace_bytes": (C.c_int32, [_P, C.POINTER(C.c_size_t)]),
    "fld_plan_bind_workspace": (C.c_int32, [_P, _P, C.c_size_t]),
    "fld_plan_levels": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "fld_plan_level_view": (C.c_int32, [_P, C.c_int32, C.c_int32, C.POINTER(fld_level_view)]),
    "fld_coefficients": (C.c_int32, [_P, _PP, _PP, C.POINTER(C.c_double), _P]),
    "fld_step": (C.c_int32, [_P, _PP, _PP, _PP, C.POINTER(C.c_double), _P, C.POINTER(fld_stats)]),
    "fld_step_noalloc": (C.c_int32, [_P, _PP, _PP, _PP, C.POINTER(C.c_double), _P, C.POINTER(fld_stats)]),
    "fld_step_aniso": (C.c_int32, [_P, _PP, _PP, _PP, C.POINTER(C.c_double), _P, C.POINTER(fld_stats)]),
    "fld_exchange": (C.c_int32, [_P, _PP, _PP, _PP, _PP, C.POINTER(C.c_double), C.POINTER(fld_gas), _P]),
    "fld_exchange_status": (C.c_int32, [_P, _P, C.POINTER(C.c_int64)]),
    "fld_plan_tuning": (C.c_int32, [_P, C.POINTER(fld_tuning)]),
    "fld_radiation_moments": (C.c_int32, [_P, _PP, _PP, _PP, C.POINTER(C.c_double), C.POINTER(fld_moments_out), _P]),
    "fld_imex_scratch_bytes": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
    "fld_imex_step": (C.c_int32, [_P, _PP, _PP, _PP, _PP, _PP, C.POINTER(C.c_double), C.POINTER(fld_gas),
                                  C.c_int32, _P, C.c_size_t, _P, C.POINTER(fld_stats)]),
    "fld_profile_kernel": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64)]),
    "fld_plan_cycle_bytes": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "fld_server_opts_default": (None, [C.POINTER(fld_server_opts)]),
    "fld_server_create": (C.c_int32, [C.POINTER(fld_server_opts), _P, C.c_size_t, _PP]),
    "fld_server_destroy": (C.c_int32, [_P]),
    "fld_submit": (C.c_int32, [_P, C.POINTER(fld_request), C.POINTER(C.c_uint64)]),
    "fld_poll": (C.c_int32, [_P, C.c_uint64, C.POINTER(fld_result)]),
    "fld_wait": (C.c_int32, [_P, C.c_uint64, C.c_double, C.POINTER(fld_result)]),
    "fld_release": (C.c_int32, [_P, C.c_uint64]),
    "fld_server_info_get": (C.c_int32, [_P, C.POINTER(fld_server_info)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class FLDError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.fld_strerror(code).decode()
        extra = _lib.fld_last_error().decode() if code == FLD_ERR_HIP else ""
        super().__init__(f"{where}: {msg} ({code}){' ' + extra if extra else ''}")
        self.code = code


def _check(code: int, where: str, ok=(FLD_OK,)) -> int:
    if code not in ok:
        raise FLDError(code, where)
    return code


def _ptrs(tensors) -> C.Array:
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t if isinstance(t, int) else t.data_ptr()
    return arr


def _dts(dt, n) -> C.Array:
    if not isinstance(dt, (list, tuple)):
        dt = [float(dt)] * n
    return (C.c_double * n)(*[float(x) for x in dt])


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---- C-named functions ----------------------------------------------------------------
def fld_version() -> int:
    return _lib.fld_version()


def fld_strerror(code: int) -> str:
    return _lib.fld_strerror(code).decode()


def fld_opts_default(**kw) -> fld_opts:
    o = fld_opts()
    _lib.fld_opts_default(C.byref(o))
    names = {f for f, _ in fld_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver option {k!r}")
        if k in ("bc", "bc_grad", "bc_value"):
            arr = getattr(o, k)
            for i, x in enumerate(v):
                arr[i] = x
        elif k == "coarse_op" and isinstance(v, str):
            o.coarse_op = COARSE_OPS[v]
        else:
            setattr(o, k, v)
    return o


def fld_gas_default(**kw) -> fld_gas:
    g = fld_gas()
    _lib.fld_gas_default(C.byref(g))
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def make_grid(n: Sequence[int], h: Optional[Sequence[float]] = None) -> fld_grid:
    """fld_grid from cell counts in x, y[, z] order (h defaults to the unit square/cube)."""
    g = fld_grid()
    g.ndim = len(n)
    for d in range(3):
        g.n[d] = int(n[d]) if d < len(n) else 1
        g.h[d] = float(h[d]) if h is not None and d < len(n) else (1.0 / max(1, n[d]) if d < len(n) else 1.0)
    return g


def fld_plan_create(grids: Sequence[fld_grid], opts: fld_opts) -> int:
    arr = (fld_grid * len(grids))(*grids)
    out = C.c_void_p()
    _check(_lib.fld_plan_create(arr, len(grids), C.byref(opts), C.byref(out)), "fld_plan_create")
    return out.value


def fld_plan_destroy(plan: int) -> None:
    _check(_lib.fld_plan_destroy(plan), "fld_plan_destroy")


def fld_plan_workspace_bytes(plan: int) -> int:
    b = C.c_size_t()
    _check(_lib.fld_plan_workspace_bytes(plan, C.byref(b)), "fld_plan_workspace_bytes")
    return b.value


def fld_plan_bind_workspace(plan: int, ptr: int, nbytes: int) -> None:
    _check(_lib.fld_plan_bind_workspace(plan, ptr, nbytes), "fld_plan_bind_workspace")


def fld_plan_levels(plan: int, g: int) -> int:
    n = C.c_int32()
    _check(_lib.fld_plan_levels(plan, g, C.byref(n)), "fld_plan_levels")
    return n.value


def fld_plan_level_view(plan: int, g: int, level: int) -> fld_level_view:
    v = fld_level_view()
    _check(_lib.fld_plan_level_view(plan, g, level, C.byref(v)), "fld_plan_level_view")
    return v


def fld_coefficients(plan: int, E_in, kappa_rho, dt, stream=None) -> None:
    n = len(E_in)
    _check(_lib.fld_coefficients(plan, _ptrs(E_in), _ptrs(kappa_rho), _dts(dt, n), _stream(stream)),
           "fld_coefficients")


def fld_step(plan: int, E_in, kappa_rho, E_out, dt, stream=None, check: bool = True):
    """Returns (status, [stats dict per grid])."""
    n = len(E_in)
    stats = (fld_stats * n)()
    rc = _lib.fld_step(plan, _ptrs(E_in), _ptrs(kappa_rho), _ptrs(E_out), _dts(dt, n),
                       _stream(stream), stats)
    if check:
        _check(rc, "fld_step")
    return rc, [s.as_dict() for s in stats]


FLD_NOALLOC_MAX_BYTES = 64 << 20


def fld_step_noalloc(plan: int, E_in, kappa_rho, E_out, dt, stream=None, check: bool = True):
    """fld_step on an unbound plan through the library's fixed device scratch (allocates
    nothing).  Returns (status, [stats dict per grid])."""
    n = len(E_in)
    stats = (fld_stats * n)()
    rc = _lib.fld_step_noalloc(plan, _ptrs(E_in), _ptrs(kappa_rho), _ptrs(E_out), _dts(dt, n),
                               _stream(stream), stats)
    if check:
        _check(rc, "fld_step_noalloc")
    return rc, [s.as_dict() for s in stats]


def fld_step_aniso(plan: int, E_in, kappa_rho_dir, E_out, dt, stream=None, check: bool = True):
    """kappa_rho_dir: per grid a list of ndim tensors (x first).  Returns (status, stats)."""
    n = len(E_in)
    kp = _vptrs(kappa_rho_dir, n)
    stats = (fld_stats * n)()
    rc = _lib.fld_step_aniso(plan, _ptrs(E_in), kp, _ptrs(E_out), _dts(dt, n), _stream(stream), stats)
    if check:
        _check(rc, "fld_step_aniso")
    return rc, [s.as_dict() for s in stats]


def fld_exchange(plan: int, E, eps, rho, kappa, dt, gas: fld_gas, stream=None) -> None:
    n = len(E)
    _check(_lib.fld_exchange(plan, _ptrs(E), _ptrs(eps), _ptrs(rho), _ptrs(kappa), _dts(dt, n),
                             C.byref(gas), _stream(stream)), "fld_exchange")


def fld_exchange_status(plan: int, stream=None):
    b = C.c_int64()
    rc = _lib.fld_exchange_status(plan, _stream(stream), C.byref(b))
    return rc, b.value


def fld_radiation_moments(plan: int, E, kappa_rho, outs, v=None, dt=None, stream=None) -> None:
    """outs: one dict per grid with optional keys F, f_r (lists of ndim tensors), edd,
    P (list of ndim (ndim+1)/2 tensors), tiring, E_out; v: per grid a list of ndim
    velocity tensors, or None."""
    n = len(E)
    arr = (fld_moments_out * n)()
    for g, o in enumerate(outs):
        ptr = lambda t: 0 if t is None else (t if isinstance(t, int) else t.data_ptr())
        for a, t in enumerate(o.get("F") or []):
            arr[g].F[a] = ptr(t)
        for a, t in enumerate(o.get("f_r") or []):
            arr[g].f_r[a] = ptr(t)
        for q, t in enumerate(o.get("P") or []):
            arr[g].P[q] = ptr(t)
        arr[g].edd = ptr(o.get("edd"))
        arr[g].tiring = ptr(o.get("tiring"))
        arr[g].E_out = ptr(o.get("E_out"))
    vp = _vptrs(v, n)
    dts = _dts(dt, n) if dt is not None else None
    _check(_lib.fld_radiation_moments(plan, _ptrs(E), _ptrs(kappa_rho), vp, dts, arr, _stream(stream)),
           "fld_radiation_moments")


def _vptrs(v, n):
    if v is None:
        return None
    vp = (C.c_void_p * (3 * n))()
    for g, comps in enumerate(v):
        for a, t in enumerate(comps or []):
            vp[3 * g + a] = 0 if t is None else t.data_ptr()
    return vp


def fld_imex_scratch_bytes(plan: int, scheme: int) -> int:
    b = C.c_size_t()
    _check(_lib.fld_imex_scratch_bytes(plan, scheme, C.byref(b)), "fld_imex_scratch_bytes")
    return b.value


def fld_imex_step(plan: int, E, eps, rho, kappa, dt, gas: fld_gas, scheme: int, scratch, scratch_bytes: int,
                  v=None, stream=None, check: bool = True):
    """In place on E and eps; returns (status, [stats dict per grid])."""
    n = len(E)
    stats = (fld_stats * n)()
    sp = scratch if isinstance(scratch, int) else (scratch.data_ptr() if scratch is not None else None)
    rc = _lib.fld_imex_step(plan, _ptrs(E), _ptrs(eps), _ptrs(rho), _ptrs(kappa), _vptrs(v, n), _dts(dt, n),
                            C.byref(gas), scheme, sp, scratch_bytes, _stream(stream), stats)
    if check:
        _check(rc, "fld_imex_step")
    return rc, [s.as_dict() for s in stats]


def fld_plan_tuning(plan: int) -> dict:
    """Launch shape of a bound plan: tile rows / width class, block cap, and its source
    (0 options, 1 timed at bind, 2 autotuner cache)."""
    t = fld_tuning()
    _check(_lib.fld_plan_tuning(plan, C.byref(t)), "fld_plan_tuning")
    return t.as_dict()


def fld_plan_cycle_bytes(plan: int, what: int = FLD_CYCLE_ITERATION):
    """Returns (algorithmic bytes, kernel launches) of one pass of a driver (host only)."""
    b = C.c_double()
    n = C.c_int64()
    _check(_lib.fld_plan_cycle_bytes(plan, what, C.byref(b), C.byref(n)), "fld_plan_cycle_bytes")
    return b.value, n.value


def fld_profile_kernel(plan: int, kernel: int, level: int = 0, reps: int = 100, stream=None):
    """Returns (mean ms per launch, cells per launch)."""
    ms = C.c_double()
    cells = C.c_int64()
    _check(_lib.fld_profile_kernel(plan, kernel, level, reps, _stream(stream), C.byref(ms), C.byref(cells)),
           "fld_profile_kernel")
    return ms.value, cells.value


def fld_server_opts_default(**kw) -> fld_server_opts:
    o = fld_server_opts()
    _lib.fld_server_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def fld_server_create(opts: fld_server_opts, arena_ptr: int, arena_bytes: int) -> int:
    out = C.c_void_p()
    _check(_lib.fld_server_create(C.byref(opts), arena_ptr, arena_bytes, C.byref(out)), "fld_server_create")
    return out.value


def fld_server_destroy(server: int) -> None:
    _check(_lib.fld_server_destroy(server), "fld_server_destroy")


def fld_submit(server: int, grid: fld_grid, dt: float, E_in, kappa_rho, on_device: bool = True,
               stream=None):
    """Returns (status, ticket).  Device inputs are read at admission, after the work
    enqueued on `stream` (default: torch's current stream) before this call."""
    req = fld_request()
    req.grid = grid
    req.dt = float(dt)
    req.E_in = E_in if isinstance(E_in, int) else (E_in.data_ptr() if on_device else
                                                   E_in.ctypes.data)
    req.kappa_rho = kappa_rho if isinstance(kappa_rho, int) else (kappa_rho.data_ptr() if on_device else
                                                                  kappa_rho.ctypes.data)
    req.inputs_on_device = 1 if on_device else 0
    req.stream = _stream(stream) if on_device else None
    t = C.c_uint64()
    rc = _lib.fld_submit(server, C.byref(req), C.byref(t))
    return rc, t.value


def fld_poll(server: int, ticket: int):
    """Returns (status, fld_result)."""
    r = fld_result()
    rc = _lib.fld_poll(server, ticket, C.byref(r))
    return rc, r


def fld_wait(server: int, ticket: int, timeout_s: float = 60.0):
    r = fld_result()
    rc = _lib.fld_wait(server, ticket, float(timeout_s), C.byref(r))
    return rc, r


def fld_release(server: int, ticket: int) -> int:
    return _lib.fld_release(server, ticket)


def fld_server_info_get(server: int) -> dict:
    i = fld_server_info()
    _check(_lib.fld_server_info_get(server, C.byref(i)), "fld_server_info_get")
    return i.as_dict()


class Server:
    """A request server over a torch-owned device arena of ``arena_bytes``."""

    def __init__(self, arena_bytes: int, device=None, **opts):
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        self.opts = fld_server_opts_default(**opts)
        self._inputs = {}
        with torch.cuda.device(self.device):
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
            self.handle = fld_server_create(self.opts, self.arena.data_ptr(), int(arena_bytes))

    def submit(self, E_in, kappa_rho, dt: float, h=None, on_device: bool = True, stream=None):
        """E_in, kappa_rho: (ny, nx) / (nz, ny, nx) float64 tensors (device) or arrays (host).

        Device tensors are read when the request is admitted, after the work enqueued on
        `stream` (default: torch's current stream) before this call; the server keeps a
        reference to them until the ticket is released."""
        shape = tuple(E_in.shape)
        grid = make_grid(tuple(reversed(shape)), h)
        rc, t = fld_submit(self.handle, grid, dt, E_in, kappa_rho, on_device, stream)
        _check(rc, "fld_submit")
        if on_device:
            self._inputs[t] = (E_in, kappa_rho)
        return t

    def result_tensor(self, res: fld_result, shape):
        """A torch view of a finished request's result buffer (inside the arena)."""
        import torch
        n = 1
        for s in shape:
            n *= s
        off = res.E_out - self.arena.data_ptr()
        return self.arena[off: off + 8 * n].view(torch.float64).view(tuple(shape))

    def wait(self, ticket: int, timeout_s: float = 60.0):
        return fld_wait(self.handle, ticket, timeout_s)

    def poll(self, ticket: int):
        return fld_poll(self.handle, ticket)

    def release(self, ticket: int):
        rc = fld_release(self.handle, ticket)
        if rc == FLD_OK:
            self._inputs.pop(ticket, None)
        return rc

    def info(self) -> dict:
        return fld_server_info_get(self.handle)

    def close(self):
        h = getattr(self, "handle", None)
        if h:
            fld_server_destroy(h)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- convenience wrapper -----------------------------------------------------------
class Plan:
    """A plan plus its torch-owned workspace.

    ``shapes`` are array shapes ((ny, nx) or (nz, ny, nx)); ``h`` per grid in x, y[, z]
    order (default: unit square / cube).
    """

    def __init__(self, shapes, h=None, device=None, **opts):
        import torch
        self.shapes = [tuple(int(s) for s in sh) for sh in shapes]
        grids = []
        for i, sh in enumerate(self.shapes):
            n = tuple(reversed(sh))
            grids.append(make_grid(n, None if h is None else h[i]))
        self.opts = fld_opts_default(**opts)
        self.device = torch.device(device if device is not None else "cuda")
        with torch.cuda.device(self.device):
            self.handle = fld_plan_create(grids, self.opts)
            nbytes = fld_plan_workspace_bytes(self.handle)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            fld_plan_bind_workspace(self.handle, self.workspace.data_ptr(), nbytes)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                fld_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def close(self):
        self.__del__()

    @property
    def ngrids(self) -> int:
        return len(self.shapes)

    def levels(self, g: int) -> int:
        return fld_plan_levels(self.handle, g)

    def level_tensors(self, g: int, level: int):
        """Views of one level's workspace arrays as torch tensors (shape (nz, ny, nx) / (ny, nx))."""
        import torch
        v = fld_plan_level_view(self.handle, g, level)
        shape = tuple(reversed([v.n[d] for d in range(v.ndim)]))
        n = 1
        for s in shape:
            n *= s
        base = self.workspace.data_ptr()

        def view(ptr, dtype, size):
            if not ptr:
                return None
            off = ptr - base
            return self.workspace[off: off + n * size].view(dtype).view(shape)

        out = {"x": view(v.x, torch.float64, 8), "b": view(v.b, torch.float64, 8),
               "x32": view(v.x32, torch.float32, 4), "b32": view(v.b32, torch.float32, 4)}
        out["w"] = [view(v.w[d], torch.float64, 8) for d in range(v.ndim)]
        out["w32"] = [view(v.w32[d], torch.float32, 4) for d in range(v.ndim)]
        out["ad"] = view(v.ad, torch.float64, 8)
        return out

    def coefficients(self, E_in, kappa_rho, dt, stream=None):
        fld_coefficients(self.handle, E_in, kappa_rho, dt, stream)

    def step(self, E_in, kappa_rho, E_out, dt, stream=None, check: bool = True):
        return fld_step(self.handle, E_in, kappa_rho, E_out, dt, stream, check)

    def step_aniso(self, E_in, kappa_rho_dir, E_out, dt, stream=None, check: bool = True):
        return fld_step_aniso(self.handle, E_in, kappa_rho_dir, E_out, dt, stream, check)

    def exchange(self, E, eps, rho, kappa, dt, gas: Optional[fld_gas] = None, stream=None):
        fld_exchange(self.handle, E, eps, rho, kappa, dt, gas or fld_gas_default(), stream)

    def exchange_status(self, stream=None):
        return fld_exchange_status(self.handle, stream)

    def imex_step(self, E, eps, rho, kappa, dt, gas: Optional[fld_gas] = None, scheme: str = "midpoint", v=None,
                  stream=None, check: bool = True):
        """One IMEX step in place on E and eps (lists of tensors per grid); the scratch
        is a torch buffer kept with the plan and grown on demand."""
        import torch
        code = IMEX_SCHEMES[scheme]
        need = fld_imex_scratch_bytes(self.handle, code)
        buf = getattr(self, "_imex_scratch", None)
        if buf is None or buf.numel() < need:
            buf = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            self._imex_scratch = buf
        return fld_imex_step(self.handle, E, eps, rho, kappa, dt, gas or fld_gas_default(c=self.opts.c), code,
                             buf.data_ptr(), buf.numel(), v=v, stream=stream, check=check)

    def profile(self, kernel: int, level: int = 0, reps: int = 100, stream=None):
        return fld_profile_kernel(self.handle, kernel, level, reps, stream)

    def tuning(self) -> dict:
        return fld_plan_tuning(self.handle)

    def cycle_bytes(self, what: int = FLD_CYCLE_ITERATION):
        return fld_plan_cycle_bytes(self.handle, what)

    def radiation_moments(self, E, kappa_rho, v=None, dt=None, want=("F", "f_r", "edd", "P"), stream=None):
        """Allocate the requested outputs (torch, on the plan's device) and run
        fld_radiation_moments; returns one dict of tensors per grid.  With v (per grid a
        list of velocity tensors) "tiring" and "E_out" may be requested as well."""
        import torch
        outs = []
        for g, e in enumerate(E):
            nd = e.dim()
            o = {}
            if "F" in want:
                o["F"] = [torch.empty_like(e) for _ in range(nd)]
            if "f_r" in want:
                o["f_r"] = [torch.empty_like(e) for _ in range(nd)]
            if "edd" in want:
                o["edd"] = torch.empty_like(e)
            if "P" in want:
                o["P"] = [torch.empty_like(e) for _ in range(nd * (nd + 1) // 2)]
            if "tiring" in want:
                o["tiring"] = torch.empty_like(e)
            if "E_out" in want:
                o["E_out"] = torch.empty_like(e)
            outs.append(o)
        fld_radiation_moments(self.handle, E, kappa_rho, outs, v=v, dt=dt, stream=stream)
        return outs
