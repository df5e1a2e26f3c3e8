"""FP64 CPU oracle for the one-domain porous-media lattice Boltzmann step (Gusev & Karlin).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the GPU library is
checked against.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product path never does.  It shares no code with the GPU
library: the arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, ``-ffp-contract=off``) and
this module only marshals numpy arrays through ctypes.

Every routine of the C file cites the section or equation of the paper it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
# LBM_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and UndefinedBehaviorSanitizer
# (host code only; the process must preload libasan, see tests/test_oracle_sanitized.py)
SANITIZE = os.environ.get("LBM_ORACLE_SANITIZE", "") == "1"
_LIB = os.path.join(_HERE, "liblbm_oracle_san.so" if SANITIZE else "liblbm_oracle.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no vectorisation-sensitive flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        extra = SANITIZE_FLAGS if SANITIZE else []
        subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("RT", ctypes.c_double), ("nu_f", ctypes.c_double), ("nu_eff_ref", ctypes.c_double),
        ("nu_eff_pow", ctypes.c_int), ("eta_eff", ctypes.c_double),
        ("b", ctypes.c_double * 3), ("rho0", ctypes.c_double),
        ("visc_corr", ctypes.c_int), ("ext_corr", ctypes.c_int), ("lagged", ctypes.c_int),
        ("eps", ctypes.POINTER(ctypes.c_double)), ("kappa", ctypes.POINTER(ctypes.c_double)),
        ("cf", ctypes.POINTER(ctypes.c_double)), ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("rho_init", ctypes.POINTER(ctypes.c_double)), ("v_init", ctypes.POINTER(ctypes.c_double)),
        ("bc_type", ctypes.POINTER(ctypes.c_uint8)), ("bc_normal", ctypes.POINTER(ctypes.c_uint8)),
        ("bc_vel", ctypes.POINTER(ctypes.c_double)), ("bc_rho", ctypes.POINTER(ctypes.c_double)),
        ("bc_scheme", ctypes.c_int), ("bc_density", ctypes.c_int),
        ("picard_iters", ctypes.c_int), ("picard_omega", ctypes.c_double),
        ("grad_eps", ctypes.POINTER(ctypes.c_double)), ("hess_eps", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Params), ctypes.c_char_p, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_time.argtypes = [ctypes.c_void_p]
        L.orc_time.restype = ctypes.c_long
        L.orc_moments.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_get_state.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_state.argtypes = [ctypes.c_void_p, dp, ctypes.c_long]
        L.orc_stats.argtypes = [ctypes.c_void_p, dp]
        L.orc_forcing_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, dp, dp]
        L.orc_delta_nu_field.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_porosity_derivatives.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_post_collision.argtypes = [ctypes.c_void_p, ctypes.c_long,
                                         ctypes.POINTER(ctypes.c_long), dp]
        L.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
        L.orc_weights.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_product_form.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc_drag_solve.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_boundary_viscous_term.argtypes = [ctypes.c_void_p, dp, ctypes.c_long,
                                                ctypes.POINTER(ctypes.c_long), dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's per-cell passes (0: the OpenMP default, OMP_NUM_THREADS or the
    core count); returns the number in use.  Results do not depend on it."""
    return int(lib().orc_set_threads(int(n)))


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(D: int):
    """Velocities c [Q,3] and opposite indices [Q] in the oracle's numbering."""
    c = (ctypes.c_int * 81)()
    opp = (ctypes.c_int * 27)()
    Q = lib().orc_lattice(D, c, opp)
    return (np.array(c[:3 * Q], dtype=np.int64).reshape(Q, 3),
            np.array(opp[:Q], dtype=np.int64))


def weights(D: int, RT: float) -> np.ndarray:
    w = np.zeros(27)
    Q = lib().orc_weights(D, RT, _dp(w))
    return w[:Q].copy()


def product_form(D: int, eps: float, rho: float, xi, P) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    f = np.zeros(27)
    lib().orc_product_form(D, eps, rho, _dp(xi), _dp(P), _dp(f))
    return f[:3 ** D].copy()


def drag_solve(v0, muD: float, muF: float) -> np.ndarray:
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    out = np.zeros_like(v0)
    lib().orc_drag_solve(len(v0), _dp(v0), muD, muF, _dp(out))
    return out


@dataclass
class OracleConfig:
    """Physical setup of one run.  Arrays are indexed [z, y, x] (x fastest)."""
    D: int
    eps: np.ndarray
    kappa: np.ndarray
    cf: np.ndarray
    mask: Optional[np.ndarray] = None
    RT: float = 1.0 / 3.0
    nu_f: float = 1.0 / 6.0
    nu_eff_ref: float = 1.0 / 6.0
    nu_eff_pow: int = 0
    eta_eff: float = math.nan
    b: tuple = (0.0, 0.0, 0.0)
    rho0: float = 1.0
    visc_corr: int = 1
    ext_corr: int = 1
    lagged: int = 0
    rho_init: Optional[np.ndarray] = None
    v_init: Optional[np.ndarray] = None   # [D, nz, ny, nx]
    # wet-node boundaries (Sec. 3.4): node type 0 bulk, 1 velocity, 2 pressure, 3 outflow;
    # outward normal 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
    bc_type: Optional[np.ndarray] = None
    bc_normal: Optional[np.ndarray] = None
    bc_vel: Optional[np.ndarray] = None    # [D, nz, ny, nx]
    bc_rho: Optional[np.ndarray] = None
    bc_scheme: int = 1                     # 0 equilibrium, 1 NEEM, 2 TMS
    bc_density: int = 0                    # 0 mass continuity, 1 bounce-back
    picard_iters: int = 0                  # App. F: Picard iterations after the one-shot step
    picard_omega: float = 1.0
    # analytic porosity derivatives (Sec. 3.5): grad eps [D, nz, ny, nx] and the Hessian's upper
    # triangle row by row [D(D+1)/2, nz, ny, nx]; None: central differences
    grad_eps: Optional[np.ndarray] = None
    hess_eps: Optional[np.ndarray] = None


class Oracle:
    """One FP64 reference run; fields are returned as numpy arrays shaped [.., nz, ny, nx]."""

    def __init__(self, cfg: OracleConfig):
        eps = np.ascontiguousarray(cfg.eps, dtype=np.float64)
        if eps.ndim == 2:
            eps = eps[None]
        self.shape = eps.shape  # (nz, ny, nx)
        nz, ny, nx = self.shape
        self.D = cfg.D
        self.N = nx * ny * nz
        self.Q = 3 ** cfg.D
        self._keep = []

        def arr(a, shape=None):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape or self.shape))
            self._keep.append(a)
            return a

        self._eps = arr(eps)
        self._kappa = arr(cfg.kappa)
        self._cf = arr(cfg.cf)
        p = _Params()
        p.D, p.nx, p.ny, p.nz = cfg.D, nx, ny, nz
        p.RT, p.nu_f, p.nu_eff_ref = cfg.RT, cfg.nu_f, cfg.nu_eff_ref
        p.nu_eff_pow, p.eta_eff = cfg.nu_eff_pow, cfg.eta_eff
        for a in range(3):
            p.b[a] = float(cfg.b[a]) if a < len(cfg.b) else 0.0
        p.rho0 = cfg.rho0
        p.visc_corr, p.ext_corr, p.lagged = cfg.visc_corr, cfg.ext_corr, cfg.lagged
        p.eps, p.kappa, p.cf = _dp(self._eps), _dp(self._kappa), _dp(self._cf)
        if cfg.mask is not None:
            m = np.ascontiguousarray(np.asarray(cfg.mask, dtype=np.uint8).reshape(self.shape))
            self._keep.append(m)
            p.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            self.mask = m.astype(bool)
        else:
            self.mask = np.zeros(self.shape, dtype=bool)
        p.rho_init = _dp(arr(cfg.rho_init))
        p.v_init = _dp(arr(cfg.v_init, (cfg.D,) + self.shape))

        def u8(a):
            if a is None:
                return ctypes.POINTER(ctypes.c_uint8)()
            a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8).reshape(self.shape))
            self._keep.append(a)
            return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

        p.bc_type, p.bc_normal = u8(cfg.bc_type), u8(cfg.bc_normal)
        p.bc_vel = _dp(arr(cfg.bc_vel, (cfg.D,) + self.shape))
        p.bc_rho = _dp(arr(cfg.bc_rho))
        p.bc_scheme, p.bc_density = cfg.bc_scheme, cfg.bc_density
        p.picard_iters, p.picard_omega = cfg.picard_iters, cfg.picard_omega
        p.grad_eps = _dp(arr(cfg.grad_eps, (cfg.D,) + self.shape))
        p.hess_eps = _dp(arr(cfg.hess_eps, (cfg.D * (cfg.D + 1) // 2,) + self.shape))
        err = ctypes.create_string_buffer(256)
        h = lib().orc_create(ctypes.byref(p), err, 256)
        if not h:
            raise ValueError("oracle create failed: " + err.value.decode())
        self._h = ctypes.c_void_p(h)
        self._params = p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib().orc_time(self._h)

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def moments(self):
        """(rho, v, v1): intrinsic density, corrected superficial velocity, drag-solve velocity."""
        rho = np.zeros(self.shape)
        v = np.zeros((self.D,) + self.shape)
        v1 = np.zeros((self.D,) + self.shape)
        lib().orc_moments(self._h, _dp(rho), _dp(v), _dp(v1))
        return rho, v, v1

    def populations(self) -> np.ndarray:
        f = np.zeros((self.Q,) + self.shape)
        lib().orc_get_state(self._h, _dp(f))
        return f

    def set_populations(self, f: np.ndarray, t: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((self.Q,) + self.shape)
        lib().orc_set_state(self._h, _dp(f), int(t))

    def stats(self) -> dict:
        out = np.zeros(8)
        lib().orc_stats(self._h, _dp(out))
        return {"mass": out[0], "momentum": out[1:4].copy(), "vmax": out[4],
                "dv2": out[5], "v2": out[6], "nonfinite": int(out[7]),
                "residual": math.sqrt(out[5] / out[6]) if out[6] > 0 else math.inf}

    def forcing_fields(self) -> dict:
        D, sh = self.D, self.shape
        acc = np.zeros((D,) + sh); phx = np.zeros((D,) + sh); pheta = np.zeros(sh)
        xi = np.zeros((D,) + sh); P = np.zeros((D,) + sh)
        xs = np.zeros((D,) + sh); Ps = np.zeros((D,) + sh)
        lib().orc_forcing_fields(self._h, _dp(acc), _dp(phx), _dp(pheta), _dp(xi), _dp(P),
                                 _dp(xs), _dp(Ps))
        return {"a": acc, "phi_ext": phx, "phi_eta": pheta, "xi": xi, "P": P,
                "xi_s": xs, "P_s": Ps}

    def delta_nu(self, m: np.ndarray) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.float64).reshape((self.D,) + self.shape)
        out = np.zeros_like(m)
        lib().orc_delta_nu_field(self._h, _dp(m), _dp(out))
        return out

    def boundary_viscous_term(self, v: np.ndarray, nodes: np.ndarray) -> np.ndarray:
        """The viscous term of eq. (accel_approx_boundary) at the given face nodes (flat cell
        indices), from the velocity field v [D, ...] (overwrites the v^(1) records)."""
        v = np.ascontiguousarray(v, dtype=np.float64).reshape((self.D,) + self.shape)
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros(len(nodes))
        lib().orc_boundary_viscous_term(self._h, _dp(v), len(nodes),
                                        nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                        _dp(out))
        return out

    def porosity_derivatives(self):
        ge = np.zeros((self.D,) + self.shape)
        H = np.zeros((self.D, self.D) + self.shape)
        lib().orc_porosity_derivatives(self._h, _dp(ge), _dp(H))
        return ge, H

    def post_collision(self, cells: np.ndarray) -> np.ndarray:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((len(cells), self.Q))
        lib().orc_post_collision(self._h, len(cells),
                                 cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out))
        return out
