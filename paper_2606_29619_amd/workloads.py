"""Seeded synthetic inputs for the porous-media lattice Boltzmann solver.

This module only builds input fields (porosity eps, permeability kappa, Forchheimer coefficient
C_F, solid mask) and run settings; it holds none of the method's arithmetic.  The tests feed the
same arrays to the GPU library and to the CPU oracle.  Arrays are shaped [nz, ny, nx] (x
fastest); two-dimensional cases use nz = 1.

Recipes (each states the workload it stands for):

* ``channel_step_2d`` -- D2Q9 FP64 128x64 channel, periodic in x, solid rows y = 0 and y = 63,
  porosity 1 for x < 64 and 0.4 for x >= 64 with permeability 1e-3 and Forchheimer coefficient
  0.55/sqrt(K) in the porous half, nu = 1/6 with nu_eff = nu/phi, body force 1e-6 along x.  The
  two porosity interfaces (x = 63.5 and the periodic seam) are smoothed with the paper's C-inf
  smoothstep over 8 cells by default, since the method needs a twice-differentiable porosity.
* ``random_porosity_3d`` -- D3Q27 periodic box with a seeded Gaussian random porosity field:
  white noise from numpy's PCG64(seed), periodic FFT filter with a Gaussian kernel whose
  covariance is exp(-r^2 / (2 l^2)) with l the correlation length (16 cells), standardised and
  mapped through the normal CDF onto phi in (phi_min, 1); Kozeny-Carman permeability
  K = d^2 phi^3 / (180 (1 - phi)^2) with d = 2 cells, C_F = 0.55 / sqrt(K); nu = 0.01; body force
  1e-6 along x.
* ``sphere_duct_3d`` -- D3Q27 duct with solid walls on the y and z faces and a porous sphere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.special import ndtr

FORCH_F = 0.55          # Forchheimer constant of the workloads: C_F = 0.55 / sqrt(K)


@dataclass
class Workload:
    """Fields and settings of one run; ``lattice`` is 9 (D2Q9) or 27 (D3Q27)."""
    name: str
    lattice: int
    eps: np.ndarray
    kappa: np.ndarray
    forch: np.ndarray
    mask: Optional[np.ndarray]
    nu_f: float
    nu_eff_ref: float
    nu_eff_pow: int
    b: tuple
    rho0: float = 1.0
    RT: float = 1.0 / 3.0
    eta_eff: float = math.nan
    steps: int = 0
    rho_init: Optional[np.ndarray] = None
    v_init: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    # wet-node boundaries: node type (0 bulk, 1 velocity, 2 pressure, 3 outflow), outward
    # normal (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z), prescribed velocity [D] and density
    bc_type: Optional[np.ndarray] = None
    bc_normal: Optional[np.ndarray] = None
    bc_velocity: Optional[np.ndarray] = None
    bc_density: Optional[np.ndarray] = None
    bc_scheme: int = 1          # 0 equilibrium, 1 NEEM, 2 TMS
    bc_rho_rule: int = 0        # 0 mass continuity, 1 bounce-back
    picard_iters: int = 0       # second-order velocity evaluation: Picard iterations
    picard_omega: float = 1.0
    # analytic porosity derivatives: grad eps [D, ...] and the Hessian's upper triangle row by
    # row [D(D+1)/2, ...] (xx, xy, yy or xx, xy, xz, yy, yz, zz); None: central differences
    grad_eps: Optional[np.ndarray] = None
    hess_eps: Optional[np.ndarray] = None

    @property
    def D(self) -> int:
        return 2 if self.lattice == 9 else 3

    @property
    def shape(self):
        return self.eps.shape

    @property
    def cells(self) -> int:
        return int(np.prod(self.eps.shape))


def kozeny_carman(phi: np.ndarray, d: float = 2.0) -> np.ndarray:
    """K = d^2 phi^3 / (180 (1 - phi)^2); phi = 1 gives +inf."""
    with np.errstate(divide="ignore"):
        return d * d * phi ** 3 / (180.0 * (1.0 - phi) ** 2)


def forchheimer(K: np.ndarray, F: float = FORCH_F) -> np.ndarray:
    """C_F = F / sqrt(K); K = +inf gives 0."""
    with np.errstate(divide="ignore"):
        return F / np.sqrt(K)


def gaussian_random_field(shape, ell: float, seed: int) -> np.ndarray:
    """Standardised periodic Gaussian random field with covariance exp(-r^2 / (2 ell^2))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal(shape)
    s = ell / math.sqrt(2.0)              # kernel width: cov of filtered noise has width ell
    ks = [np.fft.fftfreq(n) * 2.0 * math.pi for n in shape[:-1]]
    ks.append(np.fft.rfftfreq(shape[-1]) * 2.0 * math.pi)
    k2 = np.zeros([len(k) for k in ks])
    for ax, k in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = len(k)
        k2 = k2 + (k.reshape(sh)) ** 2
    axes = list(range(len(shape)))
    g = np.fft.irfftn(np.fft.rfftn(noise) * np.exp(-0.5 * k2 * s * s), s=shape, axes=axes)
    g -= g.mean()
    g /= g.std()
    return g


def random_porosity_3d(n=256, seed=0, ell=16.0, phi_min=0.3, d=2.0, nu=0.01, b=1e-6,
                       steps=1000, shape=None) -> Workload:
    shape = tuple(shape) if shape is not None else (n, n, n)
    g = gaussian_random_field(shape, ell, seed)
    phi = phi_min + (1.0 - phi_min) * ndtr(g)
    K = kozeny_carman(phi, d)
    return Workload(name=f"random-porosity D3Q27 {shape[2]}x{shape[1]}x{shape[0]} seed {seed}",
                    lattice=27, eps=phi, kappa=K, forch=forchheimer(K), mask=None,
                    nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0, b=(b, 0.0, 0.0), steps=steps,
                    meta={"seed": seed, "ell": ell, "phi_min": phi_min, "d": d})


def random_porosity_2d(nx=96, ny=64, seed=0, ell=8.0, phi_min=0.3, d=2.0, nu=0.05,
                       b=1e-6) -> Workload:
    g = gaussian_random_field((1, ny, nx), ell, seed)
    phi = phi_min + (1.0 - phi_min) * ndtr(g)
    K = kozeny_carman(phi, d)
    return Workload(name=f"random-porosity D2Q9 {nx}x{ny} seed {seed}", lattice=9, eps=phi,
                    kappa=K, forch=forchheimer(K), mask=None, nu_f=nu, nu_eff_ref=nu,
                    nu_eff_pow=0, b=(b, 0.0, 0.0), meta={"seed": seed})


def step_indicator(nx, x_step, width):
    """Porous indicator s(x) of a periodic channel that is free for x < x_step and porous for
    x >= x_step: s = 1 inside the porous half, 0 in the free half.  With width > 0 both
    interfaces (at x_step - 1/2 and at the periodic seam nx - 1/2) are smoothed with the C-inf
    smoothstep over `width` cells, each point following its nearer interface."""
    x = np.arange(nx, dtype=np.float64)
    if width <= 0:
        return (x >= x_step).astype(np.float64)

    def pdist(c):
        return np.mod(x - c + nx / 2.0, nx) - nx / 2.0

    d_up, d_down = pdist(x_step - 0.5), pdist(nx - 0.5)
    up = smoothstep_cinf(d_up / width + 0.5)
    down = smoothstep_cinf(-d_down / width + 0.5)
    return np.where(np.abs(d_up) < np.abs(d_down), up, down)


def channel_step_2d(nx=128, ny=64, x_step=64, phi_porous=0.4, K=1e-3, nu=1.0 / 6.0, g=1e-6,
                    steps=10000, smooth_width=8.0) -> Workload:
    """The porosity step of this channel is smoothed over `smooth_width` cells (0 keeps the
    literal step, which the explicit viscous correction cannot run stably).  In the transition
    eps = 1 + (phi_porous - 1) s, 1/kappa = s / K and C_F = s 0.55 / sqrt(K)."""
    s = step_indicator(nx, x_step, smooth_width)[None, None, :] * np.ones((1, ny, 1))
    eps = 1.0 + (phi_porous - 1.0) * s
    with np.errstate(divide="ignore"):
        kappa = K / s
    forch = s * (FORCH_F / math.sqrt(K))
    mask = np.zeros(eps.shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, ny - 1, :] = 1
    tag = "literal step" if smooth_width <= 0 else f"step smoothed over {smooth_width:g} cells"
    return Workload(name=f"step channel D2Q9 {nx}x{ny} ({tag})", lattice=9, eps=eps,
                    kappa=kappa, forch=forch, mask=mask, nu_f=nu, nu_eff_ref=nu,
                    nu_eff_pow=-1, b=(g, 0.0, 0.0), steps=steps,
                    meta={"smooth_width": smooth_width})


def bump(s: np.ndarray, m: int = 1) -> np.ndarray:
    """Localized bump B_m(s) = exp(1 - 1/(1 - s^m)) for s < 1, 0 for s >= 1 (eq. b_cinf)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    inner = s < 1.0
    out[inner] = np.exp(1.0 - 1.0 / (1.0 - s[inner] ** m))
    return out


def sphere_duct_3d(nx=768, ny=384, nz=384, radius=96.0, center=None, phi=0.5, K=5e-3,
                   nu=0.052, dp=1e-4, rho0=1.0, RT=1.0 / 3.0, steps=20000,
                   bump_m=None, drive="body") -> Workload:
    """Duct with solid walls on the y and z faces and a porous sphere.  drive "body": periodic
    in x, the pressure drop dp carried by an equivalent body force b_x = dp / (rho0 L_x) with
    p = rho RT.  drive "pressure": the x faces are solid layers too, and pressure nodes (Sec.
    3.4) at x = 1 and x = nx - 2 hold rho0 +- dp / (2 RT); the walls keep halfway bounce-back,
    b = 0, and the initial density falls linearly between the two.  bump_m None:
    a sharp sphere (porosity phi and permeability K inside, free fluid outside).  bump_m = m:
    the smooth inclusion of eq. (Porous_Cylinder_Profile) in 3D, eps = 1 - (1 - phi) B_m(s),
    s = r^2 / R^2, with 1/kappa = B_m(s) / K and C_F = 0.55 / sqrt(kappa) following the same
    bump (free fluid for s >= 1)."""
    center = center or (nx / 4.0, ny / 2.0, nz / 2.0)
    eps = np.empty((nz, ny, nx))
    kappa = np.empty((nz, ny, nx))
    x = np.arange(nx) + 0.5 - center[0]
    y = np.arange(ny) + 0.5 - center[1]
    for k in range(nz):                      # plane by plane: the full grid is 113 M cells
        zz = k + 0.5 - center[2]
        r2 = (x[None, :] ** 2 + y[:, None] ** 2 + zz * zz) / (radius * radius)
        if bump_m is None:
            inside = r2 < 1.0
            eps[k] = np.where(inside, phi, 1.0)
            kappa[k] = np.where(inside, K, np.inf)
        else:
            B = bump(r2, bump_m)
            eps[k] = 1.0 - (1.0 - phi) * B
            with np.errstate(divide="ignore"):
                kappa[k] = np.where(B > 0.0, K / np.where(B > 0.0, B, 1.0), np.inf)
    mask = np.zeros(eps.shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    mask[0, :, :] = 1
    mask[-1, :, :] = 1
    kind = "sharp" if bump_m is None else f"bump m={bump_m}"
    w = Workload(name=f"porous sphere ({kind}) in duct D3Q27 {nx}x{ny}x{nz}", lattice=27,
                 eps=eps, kappa=kappa, forch=forchheimer(kappa), mask=mask, nu_f=nu,
                 nu_eff_ref=nu, nu_eff_pow=0, b=(dp / (rho0 * nx), 0.0, 0.0), rho0=rho0,
                 RT=RT, steps=steps)
    if drive == "body":
        return w
    if drive != "pressure":
        raise ValueError(f"drive {drive!r}")
    drho = dp / RT
    mask[:, :, 0] = 1
    mask[:, :, -1] = 1
    bct = np.zeros(eps.shape, np.uint8)
    bcn = np.zeros(eps.shape, np.uint8)
    brho = np.full(eps.shape, rho0)
    bct[1:-1, 1:-1, 1], bcn[1:-1, 1:-1, 1] = 2, 0
    bct[1:-1, 1:-1, -2], bcn[1:-1, 1:-1, -2] = 2, 1
    brho[:, :, 1] = rho0 + drho / 2
    brho[:, :, -2] = rho0 - drho / 2
    xr = rho0 + drho / 2 - drho * (np.arange(nx) - 1.0) / (nx - 3)
    w.rho_init = np.broadcast_to(xr, eps.shape).copy()
    w.b = (0.0, 0.0, 0.0)
    w.bc_type, w.bc_normal, w.bc_density = bct, bcn, brho
    w.name = w.name.replace("in duct", "in pressure-driven duct")
    return w


def uniform_box(D=2, n=8, eps=0.5, K=0.1, cf=0.0, nu=0.05, b=(1e-4, 0.0, 0.0)) -> Workload:
    shape = (1, n, n) if D == 2 else (n, n, n)
    return Workload(name=f"uniform box D{D}", lattice=9 if D == 2 else 27,
                    eps=np.full(shape, eps), kappa=np.full(shape, K), forch=np.full(shape, cf),
                    mask=None, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0, b=tuple(b))


def smoothstep_cinf(psi: np.ndarray) -> np.ndarray:
    """C-infinity smoothstep S(psi): 0 for psi <= 0, 1 for psi >= 1, exp-ratio in between."""
    psi = np.asarray(psi, dtype=np.float64)
    out = np.where(psi >= 1.0, 1.0, 0.0)
    inner = (psi > 0.0) & (psi < 1.0)
    p = psi[inner]
    a = np.exp(-1.0 / p)
    c = np.exp(-1.0 / (1.0 - p))
    out[inner] = a / (a + c)
    return out


def smoothstep_cinf_derivatives(psi: np.ndarray):
    """First and second derivatives of S(psi).  Inside (0, 1), S = 1 / (1 + exp(-u)) with
    u = 1/(1 - psi) - 1/psi, so S' = S (1 - S) u' and S'' = S (1 - S) [(1 - 2 S) u'^2 + u''],
    u' = 1/psi^2 + 1/(1 - psi)^2, u'' = 2/(1 - psi)^3 - 2/psi^3; both vanish outside."""
    psi = np.asarray(psi, dtype=np.float64)
    d1 = np.zeros_like(psi)
    d2 = np.zeros_like(psi)
    inner = (psi > 0.0) & (psi < 1.0)
    p = psi[inner]
    S = smoothstep_cinf(p)
    u1 = 1.0 / p ** 2 + 1.0 / (1.0 - p) ** 2
    u2 = 2.0 / (1.0 - p) ** 3 - 2.0 / p ** 3
    d1[inner] = S * (1.0 - S) * u1
    d2[inner] = S * (1.0 - S) * ((1.0 - 2.0 * S) * u1 * u1 + u2)
    return d1, d2


def heterogeneous_channel_setup1(H: int, eps_bot=1.0, eps_top=0.5, phi_bot=0.1, phi_top=0.1):
    """Wall-normal two-plateau porosity with a smoothstep transition, sampled at the fluid rows
    of a channel with halfway walls at y = 0 and y = H (row j sits at y = j - 1/2)."""
    y = np.arange(1, H + 1) - 0.5
    psi = ((y / H) - phi_bot) / (1.0 - phi_top - phi_bot)
    return y, eps_bot + (eps_top - eps_bot) * smoothstep_cinf(psi)


def heterogeneous_channel_setup2(H: int, eps_ctr=0.7, eps_wall=0.3, phi_ctr=0.4, phi_wall=0.1):
    """Centerline-symmetric porosity (eq. Hetero_Channel_Setup_II_Profile): eps_ctr for
    |y/H - 1/2| <= phi_ctr/2, eps_wall for |y/H - 1/2| >= 1/2 - phi_wall, the smoothstep in
    between; sampled at the fluid rows (row j at y = j - 1/2)."""
    y = np.arange(1, H + 1) - 0.5
    psi = (np.abs(y / H - 0.5) - phi_ctr / 2.0) / (0.5 - phi_wall - phi_ctr / 2.0)
    return y, eps_ctr + (eps_wall - eps_ctr) * smoothstep_cinf(psi)


def ergun(eps: np.ndarray, dp: float):
    """Ergun permeability kappa = dp^2 eps^3 / (150 (1 - eps)^2) (eq. kappa_Ergun) and the
    Forchheimer coefficient C_F = F_eps / sqrt(kappa) with F_eps = 1.75 / sqrt(150 eps^3)
    (eq. F_eps_Ergun)."""
    eps = np.asarray(eps, dtype=np.float64)
    kappa = dp * dp * eps ** 3 / (150.0 * (1.0 - eps) ** 2)
    return kappa, 1.75 / np.sqrt(150.0 * eps ** 3) / np.sqrt(kappa)


def channel_2d(H: int, eps_rows, kappa_rows, cf_rows=None, nu=0.1, b=1e-6, nx=1) -> Workload:
    """D2Q9 channel periodic in x, solid rows y = 0 and y = H + 1 (halfway walls H apart,
    fluid row j at y = j - 1/2); the wall rows continue the porosity of their neighbours."""
    shape = (1, H + 2, nx)
    eps = np.ones(shape)
    kappa = np.full(shape, np.inf)
    cf = np.zeros(shape)
    eps[:, 1:-1, :] = np.asarray(eps_rows, dtype=np.float64).reshape(1, H, 1)
    eps[:, 0, :] = eps[:, 1, :]
    eps[:, -1, :] = eps[:, -2, :]
    kappa[:, 1:-1, :] = np.asarray(kappa_rows, dtype=np.float64).reshape(1, H, 1)
    if cf_rows is not None:
        cf[:, 1:-1, :] = np.asarray(cf_rows, dtype=np.float64).reshape(1, H, 1)
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = mask[:, -1, :] = 1
    return Workload(name=f"channel D2Q9 H={H}", lattice=9, eps=eps, kappa=kappa, forch=cf,
                    mask=mask, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0, b=(b, 0.0, 0.0))


def heterogeneous_channel_setup1_derivatives(H: int, eps_bot=1.0, eps_top=0.5, phi_bot=0.1,
                                             phi_top=0.1):
    """Analytic d eps / dy and d^2 eps / dy^2 of the Setup I porosity at the fluid rows."""
    y = np.arange(1, H + 1) - 0.5
    span = 1.0 - phi_top - phi_bot
    psi = ((y / H) - phi_bot) / span
    d1, d2 = smoothstep_cinf_derivatives(psi)
    dpsi = 1.0 / (H * span)
    return (eps_top - eps_bot) * d1 * dpsi, (eps_top - eps_bot) * d2 * dpsi * dpsi


def _upper_pairs(D):
    return [(a, b) for a in range(D) for b in range(a, D)]


def quadratic_box(D=2, n=(28, 22, 18), nu=0.05, b=(2e-4, -1e-4, 5e-5), kappa=0.5) -> Workload:
    """Closed box (one solid layer on every face) with the quadratic porosity
    eps = 0.65 + sum_a g_a u_a + sum_{a<=b} h_ab u_a u_b, u_a = (x_a - c_a) / n_a centred on the
    box, and its exact derivatives.  Central differences of a quadratic are exact, so a run with
    these analytic derivatives and one with differenced ones must agree to rounding."""
    g = (0.12, -0.08, 0.05)
    h = {(0, 0): 0.10, (0, 1): 0.07, (0, 2): -0.04, (1, 1): -0.09, (1, 2): 0.06, (2, 2): 0.05}
    dims = tuple(n[:D])
    shape = (1, dims[1], dims[0]) if D == 2 else (dims[2], dims[1], dims[0])
    grids = np.meshgrid(*[np.arange(k, dtype=np.float64) for k in shape], indexing="ij")
    xs = [grids[2], grids[1]] + ([grids[0]] if D == 3 else [])     # x, y (, z)
    u = [(xs[a] - (dims[a] - 1) / 2.0) / dims[a] for a in range(D)]
    eps = np.full(shape, 0.65)
    for a in range(D):
        eps = eps + g[a] * u[a]
    for (a, c) in _upper_pairs(D):
        eps = eps + h[(a, c)] * u[a] * u[c]
    grad = np.zeros((D,) + shape)
    for a in range(D):
        da = np.full(shape, g[a])
        for (p, q) in _upper_pairs(D):
            if p == a and q == a:
                da = da + 2.0 * h[(p, q)] * u[a]
            elif p == a:
                da = da + h[(p, q)] * u[q]
            elif q == a:
                da = da + h[(p, q)] * u[p]
        grad[a] = da / dims[a]
    hess = np.zeros((len(_upper_pairs(D)),) + shape)
    for k, (a, c) in enumerate(_upper_pairs(D)):
        hess[k] = (2.0 if a == c else 1.0) * h[(a, c)] / (dims[a] * dims[c])
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = mask[:, -1, :] = 1
    mask[:, :, 0] = mask[:, :, -1] = 1
    if D == 3:
        mask[0] = mask[-1] = 1
    return Workload(name=f"quadratic-porosity box D{D}", lattice=9 if D == 2 else 27, eps=eps,
                    kappa=np.full(shape, kappa), forch=np.full(shape, 0.55 / math.sqrt(kappa)),
                    mask=mask, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0, b=tuple(b[:3]),
                    grad_eps=grad, hess_eps=hess)


def sine_porosity(D=3, shape=(12, 16, 20), amp=0.15, nu=0.03, b=(2e-4, 0.0, 0.0),
                  nu_eff_pow=-1) -> Workload:
    """Periodic box with eps = 0.7 + amp sin(k_x x + 0.3) cos(k_y y) (sin(k_z z + 0.5) in 3D),
    k_a = 2 pi / n_a, Kozeny-Carman permeability (d = 2), and its exact derivatives."""
    shape = tuple(shape) if D == 3 else (1,) + tuple(shape[-2:])
    grids = np.meshgrid(*[np.arange(k, dtype=np.float64) for k in shape], indexing="ij")
    xs = [grids[2], grids[1]] + ([grids[0]] if D == 3 else [])
    ns = [shape[2], shape[1]] + ([shape[0]] if D == 3 else [])
    k = [2.0 * math.pi / m for m in ns]
    ph = [0.3, 0.0, 0.5]
    # factor functions and their derivatives: sin, cos, sin
    fs = [np.sin, np.cos, np.sin]
    d1 = [lambda t: np.cos(t), lambda t: -np.sin(t), lambda t: np.cos(t)]
    d2 = [lambda t: -np.sin(t), lambda t: -np.cos(t), lambda t: -np.sin(t)]
    t = [k[a] * xs[a] + ph[a] for a in range(D)]
    F = [fs[a](t[a]) for a in range(D)]
    F1 = [k[a] * d1[a](t[a]) for a in range(D)]
    F2 = [k[a] * k[a] * d2[a](t[a]) for a in range(D)]

    def prod(sel):
        out = np.full(shape, amp)
        for a in range(D):
            out = out * sel[a]
        return out

    eps = 0.7 + prod(F)
    grad = np.stack([prod([F1[c] if c == a else F[c] for c in range(D)]) for a in range(D)])
    hess = np.stack([prod([(F2[c] if a == q else F1[c]) if c in (a, q) else F[c]
                           for c in range(D)]) for (a, q) in _upper_pairs(D)])
    K = kozeny_carman(eps, 2.0)
    return Workload(name=f"sine-porosity D{D}", lattice=9 if D == 2 else 27, eps=eps, kappa=K,
                    forch=forchheimer(K), mask=None, nu_f=nu, nu_eff_ref=nu,
                    nu_eff_pow=nu_eff_pow, b=tuple(b), grad_eps=grad, hess_eps=hess)


def request_stream(n_requests=512, seed=0):
    """Serving stream: per request a seeded lattice choice, sides, phi_min and nu."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for r in range(n_requests):
        rr = np.random.Generator(np.random.PCG64(seed * 100003 + r))
        lattice = 9 if rr.random() < 0.5 else 27
        if lattice == 9:
            sides = (1, int(rr.integers(64, 1025)), int(rr.integers(64, 1025)))
        else:
            sides = tuple(int(s) for s in rr.integers(32, 193, size=3))
        reqs.append({"id": r, "seed": r, "lattice": lattice, "shape": sides,
                     "phi_min": float(rr.uniform(0.2, 0.6)), "nu": float(rr.uniform(0.005, 0.05)),
                     "arrival": float(rng.exponential(1.0))})
    t = 0.0
    for q in reqs:
        t += q["arrival"]
        q["arrival_time"] = t
    return reqs


def couette_gravity_2d(H=32, eps=0.5, Da=1e-2, nu=0.1, Gamma=1.0, V0=0.01, nx=4,
                       scheme=1, rho_rule=0):
    """Couette flow under gravity between wet-node walls (Sec. 5.1): walls at y = 0 and y = H
    (grid rows 1 and H + 1, solid rows outside) moving with -V0 and +V0, gravity -g y with
    g H / RT = Gamma, homogeneous porosity with kappa = Da H^2, mu_F = 0; initial density the
    exponential profile normalised to mean 1."""
    RT = 1.0 / 3.0
    ny = H + 3
    shape = (1, ny, nx)
    g = Gamma * RT / H
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = mask[:, -1, :] = 1
    bct = np.zeros(shape, np.uint8)
    bcn = np.zeros(shape, np.uint8)
    bct[:, 1, :] = bct[:, -2, :] = 1
    bcn[:, 1, :], bcn[:, -2, :] = 2, 3
    vel = np.zeros((2,) + shape)
    vel[0, :, 1, :], vel[0, :, -2, :] = -V0, V0
    y = np.arange(H + 1.0)
    prof = np.exp(-g * y / RT)
    rho = np.ones(shape)
    rho[:, 1:-1, :] = (prof / prof.mean())[None, :, None]
    return Workload(name=f"Couette with gravity D2Q9 H={H}", lattice=9,
                    eps=np.full(shape, float(eps)), kappa=np.full(shape, Da * H * H),
                    forch=np.zeros(shape), mask=mask, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0,
                    b=(0.0, -g, 0.0), rho_init=rho, bc_type=bct, bc_normal=bcn,
                    bc_velocity=vel, bc_scheme=scheme, bc_rho_rule=rho_rule,
                    meta={"H": H, "g": g, "V0": V0, "Da": Da})


def normal_code(sx: int = 0, sy: int = 0, sz: int = 0) -> int:
    """bc_normal value of a node whose outward normals point along the axes with s != 0 (s in
    {-1, 0, 1}): the single-normal codes 0..5 (-x, +x, -y, +y, -z, +z) for one axis, else
    64 + ax + 4 ay + 16 az with a = 1 for minus, 2 for plus, 0 for none."""
    s = (sx, sy, sz)
    if sum(1 for v in s if v) == 1:
        a = next(i for i, v in enumerate(s) if v)
        return 2 * a + (1 if s[a] > 0 else 0)
    return 64 + sum((1 if v < 0 else 2 if v > 0 else 0) << (2 * i) for i, v in enumerate(s))


def wet_box(D=2, n=(32, 8, 1), faces=None, V=0.02, rho_faces=None, nu=1.0 / 6.0, b=(0, 0, 0),
            eps=None, kappa=None, forch=None, nu_eff_pow=0, scheme=1, rho_rule=0,
            v_init=None, rho_init=None) -> Workload:
    """A box of wet-node boundaries (Sec. 3.4): n = (Lx, Ly, Lz) node spacings between the
    boundary planes of each non-periodic axis (nodes at 1 .. L + 1, solid layers at 0 and
    L + 2), or the period of a periodic one.  faces maps "x-", "x+", "y-", "y+", "z-", "z+" to
    "wall" (velocity node, v = 0), "inlet" (velocity node with the profile of the inlet, x- or
    x+ only: V times the product of the parabolas across the other non-periodic axes, zero on
    their walls), "pressure" (pressure node, density rho_faces[face]) or "periodic" (both faces
    of that axis).  Nodes on two or three faces (edges, corners) are velocity nodes with v = 0."""
    faces = dict(faces or {})
    rho_faces = dict(rho_faces or {})
    axes = "xyz"[:D]
    periodic = [faces.get(f"{a}-") == "periodic" for a in axes]
    ext = [n[i] if periodic[i] else n[i] + 3 for i in range(D)]
    nx, ny = ext[0], ext[1]
    nz = ext[2] if D == 3 else 1
    shape = (nz, ny, nx)
    mask = np.zeros(shape, np.uint8)
    bct = np.zeros(shape, np.uint8)
    bcn = np.zeros(shape, np.uint8)
    vel = np.zeros((D,) + shape)
    brho = np.ones(shape)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = [xx, yy, zz]
    sides = []
    for i in range(D):
        c = coords[i]
        if periodic[i]:
            sides.append(np.zeros(shape, int))
            continue
        mask[(c == 0) | (c == ext[i] - 1)] = 1
        sides.append(np.where(c == 1, -1, np.where(c == ext[i] - 2, 1, 0)))
    fluid = mask == 0
    # inlet profile: parabolas across the non-periodic axes other than x, zero on their walls
    prof = np.full(shape, float(V))
    for i in range(1, D):
        if not periodic[i]:
            t = (coords[i] - 1) / float(n[i])
            prof = prof * 4.0 * t * (1.0 - t)
    nsides = sum(np.abs(sd) for sd in sides)
    for idx in zip(*np.nonzero(fluid & (nsides > 0))):
        sv = [int(sd[idx]) for sd in sides] + [0] * (3 - D)
        k = sum(1 for v in sv if v)
        bcn[idx] = normal_code(*sv)
        if k > 1:
            bct[idx] = 1
            continue
        a = next(i for i, v in enumerate(sv) if v)
        face = f"{'xyz'[a]}{'-' if sv[a] < 0 else '+'}"
        kind = faces.get(face, "wall")
        if kind == "wall":
            bct[idx] = 1
        elif kind == "inlet":
            bct[idx] = 1
            vel[(0,) + idx] = prof[idx]
        elif kind == "pressure":
            bct[idx] = 2
            brho[idx] = rho_faces.get(face, 1.0)
        else:
            raise ValueError(f"face {face}: {kind}")
    e = np.ones(shape) if eps is None else np.asarray(eps, float)
    k_ = np.full(shape, np.inf) if kappa is None else np.asarray(kappa, float)
    c_ = np.zeros(shape) if forch is None else np.asarray(forch, float)
    return Workload(name=f"wet-node box D{D} {n[:D]}", lattice=9 if D == 2 else 27, eps=e,
                    kappa=k_, forch=c_, mask=mask, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=nu_eff_pow,
                    b=tuple(float(x) for x in b), rho_init=rho_init, v_init=v_init,
                    bc_type=bct, bc_normal=bcn, bc_velocity=vel, bc_density=brho,
                    bc_scheme=scheme, bc_rho_rule=rho_rule,
                    meta={"n": n[:D], "V": V, "profile": prof})


def pressure_channel(D=2, L=64, H=16, W=8, drho=1e-3, outflow=False, body=0.0, eps=None,
                     kappa=None, forch=None, nu=0.1):
    """Channel along x between solid walls (halfway bounce-back): pressure nodes at x = 1
    (rho = 1 + drho/2) and at x = L + 1 (rho = 1 - drho/2), or a zero-gradient outflow there;
    columns 0 and L + 2 solid.  D = 3 adds solid walls in z (W fluid cells wide)."""
    nx, ny = L + 3, H + 2
    nz = W + 2 if D == 3 else 1
    shape = (nz, ny, nx)
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = mask[:, -1, :] = 1
    mask[:, :, 0] = mask[:, :, -1] = 1
    if D == 3:
        mask[0] = mask[-1] = 1
    inner = (slice(1, -1) if D == 3 else slice(None), slice(1, -1))
    bct = np.zeros(shape, np.uint8)
    bcn = np.zeros(shape, np.uint8)
    bct[inner + (1,)], bcn[inner + (1,)] = 2, 0
    bct[inner + (-2,)], bcn[inner + (-2,)] = (3 if outflow else 2), 1
    brho = np.ones(shape)
    brho[..., 1] = 1 + drho / 2
    brho[..., -2] = 1 - drho / 2
    x = np.arange(nx)
    rho = np.broadcast_to((1 + drho / 2 - drho * (x - 1) / L), shape).copy()
    e = np.ones(shape) if eps is None else eps
    k = np.full(shape, np.inf) if kappa is None else kappa
    c = np.zeros(shape) if forch is None else forch
    return Workload(name=f"pressure channel D{D} {L}x{H}", lattice=9 if D == 2 else 27,
                    eps=e, kappa=k, forch=c, mask=mask, nu_f=nu, nu_eff_ref=nu, nu_eff_pow=0,
                    b=(body, 0.0, 0.0), rho_init=rho, bc_type=bct, bc_normal=bcn,
                    bc_density=brho, meta={"L": L, "H": H, "drho": drho})
