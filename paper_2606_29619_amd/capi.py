"""ctypes binding of the C ABI in ``include/lbm.h`` -- argument marshalling only.

Every function here carries the name of the C entry point it wraps and does nothing but
convert arguments; all numerical work runs in ``liblbm.so`` (HIP kernels for gfx950).  PyTorch
provides the device workspace and the stream.  Loading fails loudly when the library is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK = 0
LBM_ERR_INVALID_ARG = -1
LBM_ERR_UNSUPPORTED = -2
LBM_ERR_WORKSPACE = -3
LBM_ERR_HIP = -4
LBM_ERR_NONFINITE = -5
LBM_ERR_STATE = -6
LBM_D2Q9 = 9
LBM_D3Q27 = 27
LBM_F64 = 0
LBM_F32 = 1
LBM_F16_SHIFTED = 2
LBM_BF16_SHIFTED = 3
LBM_SHIFT_WEIGHTS = 0
LBM_SHIFT_POROUS = 1
LBM_NODE_BULK, LBM_NODE_VELOCITY, LBM_NODE_PRESSURE, LBM_NODE_OUTFLOW = 0, 1, 2, 3
LBM_NORMAL_XM, LBM_NORMAL_XP, LBM_NORMAL_YM, LBM_NORMAL_YP, LBM_NORMAL_ZM, LBM_NORMAL_ZP = range(6)


def LBM_NORMAL_AXES(sx: int, sy: int, sz: int = 0) -> int:
    """bc_normal code of a node with outward normals along every axis whose s is -1 or 1."""
    sign = lambda s: 1 if s < 0 else (2 if s > 0 else 0)  # noqa: E731
    return 64 + sign(sx) + 4 * sign(sy) + 16 * sign(sz)
LBM_BC_EQUILIBRIUM, LBM_BC_NEEM, LBM_BC_TMS = 0, 1, 2
LBM_BC_RHO_CONTINUITY, LBM_BC_RHO_BOUNCE_BACK = 0, 1
LBM_SCHEME_TWO_PASS = 0
LBM_SCHEME_LAGGED = 1
LBM_TILES_AUTO = 0
LBM_TILES_RECTANGULAR = 1
LBM_PASSES_AUTO = 0          # velocity correction inside the collision pass for large runs
LBM_PASSES_SEPARATE = 1
LBM_PASSES_FUSED = 2           # fused wherever the kernel supports the run (FP32 and FP64)
LBM_DTYPE_F64 = 0
LBM_DTYPE_F32 = 1
LBM_VELOCITY_SUPERFICIAL = 0
LBM_VELOCITY_INTRINSIC = 1

_dp = ctypes.POINTER(ctypes.c_double)


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("storage", ctypes.c_int), ("scheme", ctypes.c_int),
        ("shift", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("RT", ctypes.c_double), ("nu_f", ctypes.c_double), ("nu_eff_ref", ctypes.c_double),
        ("nu_eff_pow", ctypes.c_int), ("eta_eff", ctypes.c_double),
        ("b", ctypes.c_double * 3), ("rho0", ctypes.c_double),
        ("eps", _dp), ("kappa", _dp), ("forch", _dp),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("rho_init", _dp), ("v_init", _dp),
        ("bc_type", ctypes.POINTER(ctypes.c_uint8)), ("bc_normal", ctypes.POINTER(ctypes.c_uint8)),
        ("bc_velocity", _dp), ("bc_density", _dp),
        ("bc_scheme", ctypes.c_int), ("bc_rho_rule", ctypes.c_int),
        ("picard_iters", ctypes.c_int), ("picard_omega", ctypes.c_double),
        ("grad_eps", _dp), ("hess_eps", _dp),
        ("tiles", ctypes.c_int), ("passes", ctypes.c_int),
    ]


class lbm_stats(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("vmax", ctypes.c_double),
        ("dv2", ctypes.c_double), ("v2", ctypes.c_double), ("residual", ctypes.c_double),
        ("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64),
    ]


LBM_REQ_QUEUED = 0
LBM_REQ_ACTIVE = 1
LBM_REQ_CONVERGED = 2
LBM_REQ_CENSORED = 3
LBM_REQ_FAILED = 4
LBM_REQ_FLOOR = 5


class lbm_request_info(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64), ("state", ctypes.c_int), ("steps", ctypes.c_int64),
        ("residual", ctypes.c_double), ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("cells", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class lbm_server_stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int64), ("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
        ("finished", ctypes.c_int64), ("queued", ctypes.c_int64), ("active", ctypes.c_int64),
        ("cell_updates", ctypes.c_double), ("pool_bytes", ctypes.c_size_t),
        ("pool_used", ctypes.c_size_t), ("pool_peak", ctypes.c_size_t),
    ]


class LbmError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed ({code}): {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbm.so (built by ``__graft_entry__.build()``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.lbm_footprint.argtypes = [ctypes.POINTER(lbm_params), ctypes.POINTER(ctypes.c_size_t)]
    L.lbm_create.argtypes = [ctypes.POINTER(lbm_params), vp, ctypes.c_size_t, vp,
                             ctypes.POINTER(vp)]
    L.lbm_step.argtypes = [vp, ctypes.c_int64]
    L.lbm_step_timed.argtypes = [vp, ctypes.c_int64, _dp]
    L.lbm_moments.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
    L.lbm_residual.argtypes = [vp, ctypes.POINTER(lbm_stats)]
    L.lbm_stats_noalloc.argtypes = [vp, vp]
    L.lbm_get_populations.argtypes = [vp, vp, ctypes.c_int]
    L.lbm_set_populations.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int64]
    L.lbm_get_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_lattice_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = []
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.lbm_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int, vp,
                                    ctypes.POINTER(vp)]
    L.lbm_server_submit.argtypes = [vp, ctypes.POINTER(lbm_params), ctypes.c_double,
                                    ctypes.c_int64, ctypes.c_int, i64p]
    L.lbm_server_progress.argtypes = [vp, ctypes.c_int64, i64p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
    L.lbm_server_info.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(lbm_request_info)]
    L.lbm_server_solver.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(vp)]
    L.lbm_server_release.argtypes = [vp, ctypes.c_int64]
    L.lbm_server_get_stats.argtypes = [vp, ctypes.POINTER(lbm_server_stats)]
    L.lbm_server_destroy.argtypes = [vp]
    for name in ("lbm_footprint", "lbm_create", "lbm_step", "lbm_step_timed", "lbm_moments",
                 "lbm_residual", "lbm_get_populations", "lbm_set_populations", "lbm_get_step",
                 "lbm_lattice_info", "lbm_destroy", "lbm_server_create", "lbm_server_submit",
                 "lbm_server_progress", "lbm_server_info", "lbm_server_solver",
                 "lbm_server_release", "lbm_server_get_stats", "lbm_server_destroy"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, func: str, ok=(LBM_OK,)) -> int:
    if rc not in ok and not (func == "lbm_lattice_info" and rc > 0):
        raise LbmError(rc, func, lbm_last_error())
    return rc


def lbm_last_error() -> str:
    return load().lbm_last_error().decode()


def lbm_lattice_info(lattice: int):
    c = (ctypes.c_int * 81)()
    opp = (ctypes.c_int * 27)()
    Q = _check(load().lbm_lattice_info(lattice, c, opp), "lbm_lattice_info")
    return (np.array(c[:3 * Q], dtype=np.int64).reshape(Q, 3),
            np.array(opp[:Q], dtype=np.int64))


def lbm_footprint(p: lbm_params) -> int:
    out = ctypes.c_size_t(0)
    _check(load().lbm_footprint(ctypes.byref(p), ctypes.byref(out)), "lbm_footprint")
    return out.value


def lbm_create(p: lbm_params, workspace_ptr: int, workspace_bytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    _check(load().lbm_create(ctypes.byref(p), ctypes.c_void_p(workspace_ptr), workspace_bytes,
                             ctypes.c_void_p(stream_ptr), ctypes.byref(h)), "lbm_create")
    return h


def lbm_step(h, n: int):
    _check(load().lbm_step(h, int(n)), "lbm_step")


def lbm_step_timed(h, n: int):
    ms = (ctypes.c_double * 3)()
    _check(load().lbm_step_timed(h, int(n), ms), "lbm_step_timed")
    return [ms[0], ms[1], ms[2]]


def lbm_moments(h, rho_ptr: int, v_ptr: int, dtype: int, velocity_kind: int):
    _check(load().lbm_moments(h, ctypes.c_void_p(rho_ptr), ctypes.c_void_p(v_ptr), dtype,
                              velocity_kind), "lbm_moments")


def lbm_residual(h, allow_nonfinite: bool = False) -> lbm_stats:
    s = lbm_stats()
    ok = (LBM_OK, LBM_ERR_NONFINITE) if allow_nonfinite else (LBM_OK,)
    _check(load().lbm_residual(h, ctypes.byref(s)), "lbm_residual", ok)
    return s


def lbm_stats_noalloc(h, stats_dev_ptr: int):
    _check(load().lbm_stats_noalloc(h, stats_dev_ptr), "lbm_stats_noalloc")


def lbm_get_populations(h, dev_ptr: int, dtype: int):
    _check(load().lbm_get_populations(h, ctypes.c_void_p(dev_ptr), dtype), "lbm_get_populations")


def lbm_set_populations(h, dev_ptr: int, dtype: int, step: int):
    _check(load().lbm_set_populations(h, ctypes.c_void_p(dev_ptr), dtype, int(step)),
           "lbm_set_populations")


def lbm_get_step(h) -> int:
    s = ctypes.c_int64(0)
    _check(load().lbm_get_step(h, ctypes.byref(s)), "lbm_get_step")
    return s.value


def lbm_destroy(h):
    _check(load().lbm_destroy(h), "lbm_destroy")


def lbm_server_create(pool_ptr: int, pool_bytes: int, check_every: int, max_active: int,
                      stream_ptr: int):
    h = ctypes.c_void_p()
    _check(load().lbm_server_create(ctypes.c_void_p(pool_ptr), pool_bytes, int(check_every),
                                    int(max_active), ctypes.c_void_p(stream_ptr),
                                    ctypes.byref(h)), "lbm_server_create")
    return h


def lbm_server_submit(s, p: lbm_params, tol: float, max_steps: int,
                      floor_checks: int = 0) -> int:
    rid = ctypes.c_int64(-1)
    _check(load().lbm_server_submit(s, ctypes.byref(p), float(tol), int(max_steps),
                                    int(floor_checks), ctypes.byref(rid)), "lbm_server_submit")
    return rid.value


def lbm_server_progress(s, max_rounds: int, max_finished: int = 4096):
    ids = (ctypes.c_int64 * max(max_finished, 1))()
    n = ctypes.c_int(0)
    _check(load().lbm_server_progress(s, int(max_rounds), ids, int(max_finished),
                                      ctypes.byref(n)), "lbm_server_progress")
    return [ids[k] for k in range(min(n.value, max_finished))]


def lbm_server_info(s, rid: int) -> lbm_request_info:
    out = lbm_request_info()
    _check(load().lbm_server_info(s, int(rid), ctypes.byref(out)), "lbm_server_info")
    return out


def lbm_server_solver(s, rid: int):
    h = ctypes.c_void_p()
    _check(load().lbm_server_solver(s, int(rid), ctypes.byref(h)), "lbm_server_solver")
    return h


def lbm_server_release(s, rid: int):
    _check(load().lbm_server_release(s, int(rid)), "lbm_server_release")


def lbm_server_get_stats(s) -> lbm_server_stats:
    out = lbm_server_stats()
    _check(load().lbm_server_get_stats(s, ctypes.byref(out)), "lbm_server_get_stats")
    return out


def lbm_server_destroy(s):
    _check(load().lbm_server_destroy(s), "lbm_server_destroy")


# --------------------------------------------------------------------------------------------
# Convenience wrapper: numpy fields in, torch device memory and stream underneath.
# --------------------------------------------------------------------------------------------
def make_params(lattice: int, storage: int, eps: np.ndarray, kappa: np.ndarray,
                forch: np.ndarray, mask: Optional[np.ndarray] = None, RT: float = 1.0 / 3.0,
                nu_f: float = 1.0 / 6.0, nu_eff_ref: float = 1.0 / 6.0, nu_eff_pow: int = 0,
                eta_eff: float = math.nan, b=(0.0, 0.0, 0.0), rho0: float = 1.0,
                rho_init: Optional[np.ndarray] = None, v_init: Optional[np.ndarray] = None,
                scheme: int = LBM_SCHEME_TWO_PASS, shift: int = LBM_SHIFT_WEIGHTS,
                bc_type: Optional[np.ndarray] = None, bc_normal: Optional[np.ndarray] = None,
                bc_velocity: Optional[np.ndarray] = None,
                bc_density: Optional[np.ndarray] = None, bc_scheme: int = LBM_BC_NEEM,
                bc_rho_rule: int = LBM_BC_RHO_CONTINUITY, picard_iters: int = 0,
                picard_omega: float = 1.0, grad_eps: Optional[np.ndarray] = None,
                hess_eps: Optional[np.ndarray] = None, tiles: int = LBM_TILES_AUTO,
                passes: int = LBM_PASSES_AUTO):
    """Build an lbm_params from numpy arrays shaped [nz, ny, nx]; returns (params, keepalive).
    grad_eps [D][nz, ny, nx] and hess_eps [D(D+1)/2][nz, ny, nx] (upper triangle row by row)
    are the optional analytic porosity derivatives."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    if eps.ndim == 2:
        eps = eps[None]
    nz, ny, nx = eps.shape
    keep = [eps]

    def arr(a, shape):
        if a is None:
            return _dp()
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
        keep.append(a)
        return a.ctypes.data_as(_dp)

    p = lbm_params()
    p.lattice, p.storage, p.scheme, p.shift = lattice, storage, scheme, shift
    p.nx, p.ny, p.nz = nx, ny, nz
    p.RT, p.nu_f, p.nu_eff_ref, p.nu_eff_pow, p.eta_eff = RT, nu_f, nu_eff_ref, nu_eff_pow, eta_eff
    for a in range(3):
        p.b[a] = float(b[a]) if a < len(b) else 0.0
    p.rho0 = rho0
    p.eps = eps.ctypes.data_as(_dp)
    p.kappa = arr(kappa, eps.shape)
    p.forch = arr(forch, eps.shape)
    if mask is not None:
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(eps.shape))
        keep.append(m)
        p.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    D = 2 if lattice == LBM_D2Q9 else 3
    p.rho_init = arr(rho_init, eps.shape)
    p.v_init = arr(v_init, (D,) + eps.shape)

    def u8(a):
        if a is None:
            return ctypes.POINTER(ctypes.c_uint8)()
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8).reshape(eps.shape))
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

    p.bc_type, p.bc_normal = u8(bc_type), u8(bc_normal)
    p.bc_velocity = arr(bc_velocity, (D,) + eps.shape)
    p.bc_density = arr(bc_density, eps.shape)
    p.bc_scheme, p.bc_rho_rule = bc_scheme, bc_rho_rule
    p.picard_iters, p.picard_omega = picard_iters, picard_omega
    p.grad_eps = arr(grad_eps, (D,) + eps.shape)
    p.hess_eps = arr(hess_eps, (D * (D + 1) // 2,) + eps.shape)
    p.tiles = tiles
    p.passes = passes
    return p, keep


class Solver:
    """A solver on one GPU: owns its torch workspace, uses torch's current stream."""

    def __init__(self, params: lbm_params, keepalive=None, device="cuda", handle=None):
        import torch
        self._torch = torch
        self.params = params
        self.D = 2 if params.lattice == LBM_D2Q9 else 3
        self.Q = params.lattice
        self.shape = (params.nz, params.ny, params.nx)
        self.N = params.nx * params.ny * params.nz
        # dtype of exported populations and moments: the arithmetic type
        self.dtype = torch.float64 if params.storage == LBM_F64 else torch.float32
        self.nbytes = lbm_footprint(params)
        self.device = torch.device(device)
        self._owned = handle is None
        if handle is None:
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            self._h = lbm_create(params, self.workspace.data_ptr(), self.nbytes,
                                 self.stream.cuda_stream)
        else:  # a handle owned elsewhere (a request of a server)
            self._h = handle
        del keepalive

    @classmethod
    def from_workload(cls, w, storage: int = LBM_F32, scheme: int = LBM_SCHEME_TWO_PASS,
                      shift: int = LBM_SHIFT_WEIGHTS, tiles: int = LBM_TILES_AUTO,
                      passes: int = LBM_PASSES_AUTO, **kw):
        p, keep = make_params(w.lattice, storage, w.eps, w.kappa, w.forch, w.mask, RT=w.RT,
                              nu_f=w.nu_f, nu_eff_ref=w.nu_eff_ref, nu_eff_pow=w.nu_eff_pow,
                              eta_eff=w.eta_eff, b=w.b, rho0=w.rho0, rho_init=w.rho_init,
                              v_init=w.v_init, scheme=scheme, shift=shift,
                              bc_type=getattr(w, "bc_type", None),
                              bc_normal=getattr(w, "bc_normal", None),
                              bc_velocity=getattr(w, "bc_velocity", None),
                              bc_density=getattr(w, "bc_density", None),
                              bc_scheme=getattr(w, "bc_scheme", LBM_BC_NEEM),
                              bc_rho_rule=getattr(w, "bc_rho_rule", LBM_BC_RHO_CONTINUITY),
                              picard_iters=getattr(w, "picard_iters", 0),
                              picard_omega=getattr(w, "picard_omega", 1.0),
                              grad_eps=getattr(w, "grad_eps", None),
                              hess_eps=getattr(w, "hess_eps", None), tiles=tiles,
                              passes=passes)
        return cls(p, keep, **kw)

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def step_count(self) -> int:
        return lbm_get_step(self._h)

    def step(self, n: int = 1):
        lbm_step(self._h, n)

    def step_timed(self, n: int = 1):
        return lbm_step_timed(self._h, n)

    def moments(self, dtype=None, intrinsic: bool = False):
        torch = self._torch
        dtype = dtype or torch.float64
        rho = torch.empty(self.shape, dtype=dtype, device=self.device)
        v = torch.empty((self.D,) + self.shape, dtype=dtype, device=self.device)
        code = LBM_DTYPE_F64 if dtype == torch.float64 else LBM_DTYPE_F32
        lbm_moments(self._h, rho.data_ptr(), v.data_ptr(), code,
                    LBM_VELOCITY_INTRINSIC if intrinsic else LBM_VELOCITY_SUPERFICIAL)
        return rho, v

    def populations(self, dtype=None):
        torch = self._torch
        dtype = dtype or self.dtype
        out = torch.empty((self.Q,) + self.shape, dtype=dtype, device=self.device)
        lbm_get_populations(self._h, out.data_ptr(),
                            LBM_DTYPE_F64 if dtype == torch.float64 else LBM_DTYPE_F32)
        return out

    def set_populations(self, f, step: int = 0):
        torch = self._torch
        f = f.contiguous()
        lbm_set_populations(self._h, f.data_ptr(),
                            LBM_DTYPE_F64 if f.dtype == torch.float64 else LBM_DTYPE_F32, step)
        self._keep_state = f

    def residual(self, allow_nonfinite: bool = False) -> lbm_stats:
        return lbm_residual(self._h, allow_nonfinite)


class Server:
    """A request server on one GPU: owns its device pool (a torch tensor), uses torch's current
    stream.  Marshalling only; admission, batching and retirement run in the library."""

    def __init__(self, pool_bytes: int, check_every: int = 100, max_active: int = 0,
                 device="cuda"):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.check_every = check_every
        self._params = {}
        self._h = lbm_server_create(self.pool.data_ptr(), int(pool_bytes), check_every,
                                    max_active, self.stream.cuda_stream)

    def submit_params(self, params: lbm_params, tol: float, max_steps: int,
                      floor_checks: int = 0) -> int:
        rid = lbm_server_submit(self._h, params, tol, max_steps, floor_checks)
        self._params[rid] = params
        return rid

    def submit(self, w, storage: int = LBM_F32, tol: float = 1e-7, max_steps: int = 200000,
               scheme: int = LBM_SCHEME_TWO_PASS, shift: int = LBM_SHIFT_POROUS,
               floor_checks: int = 0) -> int:
        p, _keep = make_params(w.lattice, storage, w.eps, w.kappa, w.forch, w.mask, RT=w.RT,
                               nu_f=w.nu_f, nu_eff_ref=w.nu_eff_ref, nu_eff_pow=w.nu_eff_pow,
                               eta_eff=w.eta_eff, b=w.b, rho0=w.rho0, rho_init=w.rho_init,
                               v_init=w.v_init, scheme=scheme, shift=shift,
                              bc_type=getattr(w, "bc_type", None),
                              bc_normal=getattr(w, "bc_normal", None),
                              bc_velocity=getattr(w, "bc_velocity", None),
                              bc_density=getattr(w, "bc_density", None),
                              bc_scheme=getattr(w, "bc_scheme", LBM_BC_NEEM),
                              bc_rho_rule=getattr(w, "bc_rho_rule", LBM_BC_RHO_CONTINUITY),
                              picard_iters=getattr(w, "picard_iters", 0),
                              picard_omega=getattr(w, "picard_omega", 1.0),
                              grad_eps=getattr(w, "grad_eps", None),
                              hess_eps=getattr(w, "hess_eps", None))
        rid = self.submit_params(p, tol, max_steps, floor_checks)  # the library copies the arrays
        return rid

    def progress(self, max_rounds: int = 1):
        return lbm_server_progress(self._h, max_rounds)

    def info(self, rid: int) -> lbm_request_info:
        return lbm_server_info(self._h, rid)

    def solver(self, rid: int) -> Solver:
        """A Solver view of a request (moments, populations) valid until release."""
        return Solver(self._params[rid], handle=lbm_server_solver(self._h, rid),
                      device=self.device)

    def release(self, rid: int):
        lbm_server_release(self._h, rid)

    def stats(self) -> lbm_server_stats:
        return lbm_server_get_stats(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lbm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
