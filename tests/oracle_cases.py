"""Small setups shared by the oracle pins and the GPU parity tests (inputs only, no method
arithmetic): channels with halfway walls, uniform boxes and the linear-wave setups of the
paper's dissipation study (Sec. 4.2)."""
import math

import numpy as np

import oracle
from paper_2606_29619_amd import workloads


def channel(D, H, eps_rows, kappa_rows, cf_rows=None, nu=0.1, nu_f=None, b=1e-6, pow_=0,
            visc_corr=1, ext_corr=1, nx=1, nz=1, lagged=0, deps_rows=None, d2eps_rows=None):
    """Channel periodic in x (and z), solid rows y = 0 and y = H + 1, so the halfway walls sit at
    distance H apart and fluid row j lies at y = j - 1/2 from the lower wall.  deps_rows and
    d2eps_rows: analytic d eps/dy and d^2 eps/dy^2 of the fluid rows (else differences)."""
    ny = H + 2
    shape = (nz if D == 3 else 1, ny, nx)
    eps = np.ones(shape)
    kappa = np.full(shape, np.inf)
    cf = np.zeros(shape)
    eps[:, 1:-1, :] = np.asarray(eps_rows).reshape(1, H, 1)
    eps[:, 0, :] = eps[:, 1, :]          # smooth continuation into the wall rows
    eps[:, -1, :] = eps[:, -2, :]
    kappa[:, 1:-1, :] = np.asarray(kappa_rows).reshape(1, H, 1)
    if cf_rows is not None:
        cf[:, 1:-1, :] = np.asarray(cf_rows).reshape(1, H, 1)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    grad = hess = None
    if deps_rows is not None:
        grad = np.zeros((D,) + shape)
        hess = np.zeros((D * (D + 1) // 2,) + shape)
        grad[1][:, 1:-1, :] = np.asarray(deps_rows).reshape(1, H, 1)
        hess[D][:, 1:-1, :] = np.asarray(d2eps_rows).reshape(1, H, 1)   # the yy entry
    cfg = oracle.OracleConfig(D=D, eps=eps, kappa=kappa, cf=cf, mask=mask,
                              nu_f=nu if nu_f is None else nu_f, nu_eff_ref=nu,
                              nu_eff_pow=pow_, b=(b, 0.0, 0.0), visc_corr=visc_corr,
                              ext_corr=ext_corr, lagged=lagged, grad_eps=grad, hess_eps=hess)
    return oracle.Oracle(cfg)


def run_to_steady(o, tol=1e-11, chunk=200, max_steps=200000):
    """Step until the relative L2 change of v over one chunk falls below tol."""
    o.stats()
    steps = 0
    while steps < max_steps:
        o.step(chunk)
        steps += chunk
        s = o.stats()
        if s["residual"] < tol:
            return steps
    raise AssertionError(f"no steady state after {steps} steps (residual {s['residual']:.3e})")


def profile(o):
    rho, v, _ = o.moments()
    return rho[0, 1:-1, 0], v[0, 0, 1:-1, 0]


def wave_setup(setup, L=48, JT=1.0, Ma0=0.1, Jnu=1.0, Jeta=None, ext=1, eps=0.5, nu_f=0.01):
    """Linear plane-wave setups (I)-(IV) of Sec. 4.2 with the viscous-drag-balance drag
    parameters (VDB_params); the drag is scaled with the wave's own |k|^2.  Returns the oracle
    and the analytic decay rate."""
    cfg, rate = wave_config(setup, L, JT, Ma0, Jnu, Jeta, ext, eps, nu_f)
    return oracle.Oracle(cfg), rate


def wave_config(setup, L=48, JT=1.0, Ma0=0.1, Jnu=1.0, Jeta=None, ext=1, eps=0.5, nu_f=0.01):
    """The OracleConfig of a wave setup and its analytic decay rate."""
    RT = JT / 3.0
    k = 2 * math.pi / L
    kk = 2 * k * k if setup == "III" else k * k
    muD = nu_f * kk
    muF = nu_f * kk / (eps * math.sqrt(RT))
    kappa, cf = eps * nu_f / muD, muF / eps
    y, x = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    a0 = 1e-5
    U = eps * Ma0 * math.sqrt(RT)
    v = np.zeros((2, 1, L, L))
    bmag = muD * Ma0 * math.sqrt(RT) + muF * eps * Ma0 ** 2 * RT
    if setup == "I":
        v[0, 0], v[1, 0], b = a0 * np.sin(k * y), U, (0.0, bmag, 0.0)
    elif setup == "II":
        v[0, 0], b = U + a0 * np.sin(k * x), (bmag, 0.0, 0.0)
    elif setup == "III":
        s = a0 * np.sin(k * (x + y))
        v[0, 0], v[1, 0] = (U + s) / math.sqrt(2), (U - s) / math.sqrt(2)
        bb = Ma0 / math.sqrt(2) * (muD * math.sqrt(RT) + muF * eps * Ma0 * RT)
        b = (bb, bb, 0.0)
    else:
        v[0, 0], v[1, 0], b = a0 * np.sin(k * x), U, (0.0, bmag, 0.0)
    shape = (1, L, L)
    cfg = oracle.OracleConfig(
        D=2, eps=np.full(shape, eps), kappa=np.full(shape, kappa), cf=np.full(shape, cf),
        RT=RT, nu_f=nu_f, nu_eff_ref=Jnu * nu_f, nu_eff_pow=0,
        eta_eff=math.nan if Jeta is None else Jeta * nu_f, b=b, ext_corr=ext, v_init=v)
    Jeta_eff = Jnu if Jeta is None else Jeta       # without Phi^eta the bulk viscosity is nu
    pref = 2 * math.pi ** 2 * nu_f / L ** 2
    rate = {"I": 2 * pref * (Jnu + 1 + Ma0), "II": pref * (Jnu + Jeta_eff + 1 + 2 * Ma0),
            "III": 4 * pref * (Jnu + 1 + Ma0), "IV": pref * (Jnu + Jeta_eff + 1 + Ma0)}[setup]
    return cfg, rate


def measure_decay(o, setup, steps, L):
    """Decay rate from the Fourier amplitude of vorticity (shear) or divergence (acoustic)
    computed by central differences, as in Sec. 4.2; acoustic rates from the peak envelope."""
    amps = []
    for _ in range(steps):
        _, v, _ = o.moments()
        vx, vy = v[0, 0], v[1, 0]
        dx = lambda f: (np.roll(f, -1, 1) - np.roll(f, 1, 1)) / 2
        dy = lambda f: (np.roll(f, -1, 0) - np.roll(f, 1, 0)) / 2
        q = dx(vy) - dy(vx) if setup in ("I", "III") else dx(vx) + dy(vy)
        F = np.fft.fft2(q) / (L * L)
        amps.append(abs({"I": F[1, 0], "III": F[1, 1]}.get(setup, F[0, 1])))
        o.step(1)
    amps = np.array(amps)
    t = np.arange(steps)
    if setup in ("I", "III"):
        return -np.polyfit(t[100:], np.log(amps[100:]), 1)[0]
    pk = np.array([i for i in range(1, steps - 1) if amps[i] > amps[i - 1] and amps[i] >= amps[i + 1]])
    return -np.polyfit(t[pk], np.log(amps[pk]), 1)[0]


def wall_channel(D, H, eps, kappa, nu, b, v_bot, v_top, scheme=1, density=0, nx=4, nz=1,
                 rho_init=None, cf=0.0):
    """Channel periodic in x (and z) between two wet-node walls (Sec. 3.4) at y = 0 and y = H
    (grid rows 1 and H + 1; rows 0 and H + 2 are solid), walls moving along x with v_bot and
    v_top.  Node j of the channel lies at y = j."""
    ny = H + 3
    shape = (nz if D == 3 else 1, ny, nx)
    e = np.full(shape, float(eps))
    k = np.full(shape, float(kappa))
    c = np.full(shape, float(cf))
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    bct = np.zeros(shape, np.uint8)
    bcn = np.zeros(shape, np.uint8)
    bct[:, 1, :] = 1
    bct[:, -2, :] = 1
    bcn[:, 1, :] = 2       # outward normal -y
    bcn[:, -2, :] = 3      # outward normal +y
    vel = np.zeros((D,) + shape)
    vel[0, :, 1, :] = v_bot
    vel[0, :, -2, :] = v_top
    rinit = None
    if rho_init is not None:
        rinit = np.ones(shape)
        rinit[:, 1:-1, :] = np.asarray(rho_init).reshape(1, H + 1, 1)
    cfg = oracle.OracleConfig(D=D, eps=e, kappa=k, cf=c, mask=mask, nu_f=nu, nu_eff_ref=nu,
                              b=tuple(b) + (0.0,) * (3 - len(b)), rho_init=rinit,
                              bc_type=bct, bc_normal=bcn, bc_vel=vel, bc_scheme=scheme,
                              bc_density=density)
    return oracle.Oracle(cfg)


def wall_profile(o):
    """(rho, v_x) along the channel nodes y = 0..H."""
    rho, v, _ = o.moments()
    return rho[0, 1:-1, 0], v[0, 0, 1:-1, 0]


def from_workload(w, **extra):
    """An oracle for a workload of paper_2606_29619_amd.workloads (every field it carries)."""
    cfg = oracle.OracleConfig(D=w.D, eps=w.eps, kappa=w.kappa, cf=w.forch, mask=w.mask,
                              RT=w.RT, nu_f=w.nu_f, nu_eff_ref=w.nu_eff_ref,
                              nu_eff_pow=w.nu_eff_pow, eta_eff=w.eta_eff, b=w.b, rho0=w.rho0,
                              rho_init=w.rho_init, v_init=w.v_init, bc_type=w.bc_type,
                              bc_normal=w.bc_normal, bc_vel=w.bc_velocity, bc_rho=w.bc_density,
                              bc_scheme=w.bc_scheme, bc_density=w.bc_rho_rule, **extra)
    return oracle.Oracle(cfg)
