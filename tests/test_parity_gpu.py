"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the same
seeded inputs, element by element.

FP64 storage must match to 1e-12 normwise per field, e(X) = max|X_gpu - X_orc| / max|X_orc|,
for X in {f-bar (all i), rho, rho - rho0, each component of v}.  Both sides evaluate every
expression in the same order without contraction, so the measured differences are zero or a
few ulps.  FP32 storage is compared with the tolerances derived in the test of each case.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_29619_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
capi = pytest.importorskip("paper_2606_29619_amd.capi")

FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    capi.load()
    yield
    torch.cuda.synchronize()


def _oracle_for(w, **extra):
    cfg = oracle.OracleConfig(D=w.D, eps=w.eps, kappa=w.kappa, cf=w.forch, mask=w.mask,
                              RT=w.RT, nu_f=w.nu_f, nu_eff_ref=w.nu_eff_ref,
                              nu_eff_pow=w.nu_eff_pow, eta_eff=w.eta_eff, b=w.b, rho0=w.rho0,
                              rho_init=w.rho_init, v_init=w.v_init, bc_type=w.bc_type,
                              bc_normal=w.bc_normal, bc_vel=w.bc_velocity, bc_rho=w.bc_density,
                              bc_scheme=w.bc_scheme, bc_density=w.bc_rho_rule, **extra)
    return oracle.Oracle(cfg)


def _rel(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def _field_errors(s, o, rho0=1.0):
    f_gpu = s.populations(torch.float64).cpu().numpy()
    rho_gpu, v_gpu = (t.cpu().numpy() for t in s.moments(torch.float64))
    f_ref = o.populations()
    rho_ref, v_ref, _ = o.moments()
    errs = {"f": _rel(f_gpu, f_ref), "rho": _rel(rho_gpu, rho_ref)}
    fluid = ~o.mask
    errs["rho-rho0"] = _rel(np.where(fluid, rho_gpu - rho0, 0), np.where(fluid, rho_ref - rho0, 0))
    for a in range(v_ref.shape[0]):
        errs[f"v{a}"] = _rel(v_gpu[a], v_ref[a])
    return errs


def _print(tag, errs):
    print(tag, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)


def _run_pair(w, steps, storage=capi.LBM_F64, chunks=1, lagged=False, shift=capi.LBM_SHIFT_WEIGHTS):
    scheme = capi.LBM_SCHEME_LAGGED if lagged else capi.LBM_SCHEME_TWO_PASS
    s = capi.Solver.from_workload(w, storage=storage, scheme=scheme, shift=shift)
    o = _oracle_for(w, lagged=int(lagged))
    per = steps // chunks
    for _ in range(chunks):
        s.step(per)
        o.step(per)
    torch.cuda.synchronize()
    return s, o


# --------------------------------------------------------------------------------------------
# FP64 bit-level parity
# --------------------------------------------------------------------------------------------
def test_d2q9_step_channel_full_run():
    """The D2Q9 FP64 128x64 step channel (periodic in x, solid rows y = 0 and 63, porosity 1 /
    0.4 with K = 1e-3, nu_eff = nu/phi, g = 1e-6; porosity step smoothed over 8 cells) over its
    full 10,000 steps."""
    w = workloads.channel_step_2d()
    s, o = _run_pair(w, 10000)
    errs = _field_errors(s, o)
    _print("d2q9 channel 10k:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    st = s.residual()
    assert st.nonfinite == 0 and st.step == 10000


def test_d2q9_literal_step_parity_and_blowup_detection():
    """With the literal (unsmoothed) porosity step the explicit viscous correction meets
    d eps = 0.3 and a Hessian of 0.6 at the interface: the first steps still agree to FP64
    parity (large Delta_nu terms exercised), and the run then diverges on both sides within a
    few tens of steps, which lbm_residual reports as LBM_ERR_NONFINITE."""
    w = workloads.channel_step_2d(smooth_width=0)
    s, o = _run_pair(w, 6)
    errs = _field_errors(s, o)
    _print("d2q9 literal step 6 steps:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    s.step(60)
    with pytest.raises(capi.LbmError) as ei:
        s.residual()
    assert ei.value.code == capi.LBM_ERR_NONFINITE
    st = s.residual(allow_nonfinite=True)
    assert st.nonfinite > 0


@pytest.mark.parametrize("shape,solids", [((9, 13, 70), True), ((7, 5, 130), False),
                                          ((1, 3, 1), False)])
def test_d3q27_heterogeneous_ragged(shape, solids):
    """D3Q27 FP64 on ragged shapes (x not a multiple of the 64-wide block, y not a multiple of
    4), random porosity, with and without solid blocks touching each other and the
    periodic seams."""
    w = workloads.random_porosity_3d(shape=shape, seed=11, ell=2.5, nu=0.04, b=3e-4)
    if solids:
        m = np.zeros(shape, np.uint8)
        m[2:5, 3:7, 10:20] = 1
        m[:, 0, 40:45] = 1
        m[0, :, 63:66] = 1
        w.mask = m
    s, o = _run_pair(w, 24, chunks=2)
    errs = _field_errors(s, o)
    _print(f"d3q27 {shape} solids={solids}:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


def test_d2q9_all_options():
    """D2Q9 FP64 with every option of the method switched on: RT != 1/3 (extended equilibrium
    correction active), bulk viscosity (Phi^eta), nu_eff = nu_ref eps, an initial velocity and
    density field, Forchheimer drag, solids."""
    w = workloads.random_porosity_2d(nx=67, ny=29, seed=4, ell=4.0, nu=0.03, b=2e-4)
    w.RT = 0.25
    w.eta_eff = 0.05
    w.nu_eff_pow = 1
    y, x = np.meshgrid(np.arange(29), np.arange(67), indexing="ij")
    w.v_init = np.stack([0.01 * np.sin(2 * np.pi * y / 29), 0.005 * np.cos(2 * np.pi * x / 67)])[:, None]
    w.rho_init = (1 + 0.002 * np.cos(2 * np.pi * x / 67))[None]
    m = np.zeros(w.shape, np.uint8)
    m[0, 10:14, 20:31] = 1
    w.mask = m
    s, o = _run_pair(w, 40, chunks=2)
    errs = _field_errors(s, o)
    _print("d2q9 options:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


def test_d3q27_nu_over_eps_with_eta():
    w = workloads.random_porosity_3d(shape=(6, 8, 10), seed=3, ell=2.0, nu=0.02, b=1e-4)
    w.nu_eff_pow = -1
    w.eta_eff = 0.01
    w.RT = 0.4
    s, o = _run_pair(w, 10)
    errs = _field_errors(s, o)
    _print("d3q27 nu/eps eta:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


def test_initial_state_matches():
    """Step 0: the initial populations of eq. (eq_bc_f_bar)."""
    w = workloads.random_porosity_3d(shape=(5, 6, 7), seed=9, ell=2.0, nu=0.03, b=1e-3)
    s, o = _run_pair(w, 0)
    errs = _field_errors(s, o)
    assert max(errs.values()) <= FP64_TOL, errs


# --------------------------------------------------------------------------------------------
# Lagged single-pass scheme
# --------------------------------------------------------------------------------------------
def _options_2d():
    w = workloads.random_porosity_2d(nx=67, ny=29, seed=4, ell=4.0, nu=0.03, b=2e-4)
    w.RT = 0.25
    w.eta_eff = 0.05
    w.nu_eff_pow = 1
    y, x = np.meshgrid(np.arange(29), np.arange(67), indexing="ij")
    w.v_init = np.stack([0.01 * np.sin(2 * np.pi * y / 29), 0.005 * np.cos(2 * np.pi * x / 67)])[:, None]
    w.rho_init = (1 + 0.002 * np.cos(2 * np.pi * x / 67))[None]
    m = np.zeros(w.shape, np.uint8)
    m[0, 10:14, 20:31] = 1
    w.mask = m
    return w


def _solids_3d(shape=(9, 13, 70)):
    w = workloads.random_porosity_3d(shape=shape, seed=11, ell=2.5, nu=0.04, b=3e-4)
    w.eta_eff = 0.02
    m = np.zeros(shape, np.uint8)
    m[2:5, 3:7, 10:20] = 1
    m[:, 0, 40:45] = 1
    m[0, :, 63:66] = 1
    w.mask = m
    return w


@pytest.mark.parametrize("case", ["d2q9_options", "d3q27_solids"])
def test_lagged_scheme_matches_oracle(case):
    """LBM_SCHEME_LAGGED against the oracle's lagged mode, FP64: the single fused kernel (own
    moments current, stencil neighbours from the previous step, history double-buffered) and
    the lagged velocity correction of lbm_moments, with every option and solid cells."""
    w = _options_2d() if case == "d2q9_options" else _solids_3d()
    s, o = _run_pair(w, 30, chunks=3, lagged=True)
    errs = _field_errors(s, o)
    _print(f"lagged {case}:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    # the lagged and two-pass transients differ by far more than the tolerance
    t = capi.Solver.from_workload(w, storage=capi.LBM_F64)
    t.step(30)
    _, v_two = t.moments(torch.float64)
    _, v_lag = s.moments(torch.float64)
    assert _rel(v_lag.cpu().numpy(), v_two.cpu().numpy()) > 1e-9


@pytest.mark.parametrize("D,lagged,storage", [(3, False, "f64"), (3, True, "f64"),
                                               (2, False, "f64"), (3, False, "f16")])
def test_solid_free_tiles_match_oracle(D, lagged, storage):
    """A large domain whose few solid cells sit in one corner region and one thin wall: most
    workgroup tiles have no solid cell within one cell and take the solid-free code, the others
    the solid-aware code, in one launch.  FP64 must still match the oracle to 1e-12 (both AA
    phases at the checks); FP16 storage (porous shift) stays within its bulk bounds."""
    if D == 3:
        shape = (6, 24, 300)
        w = workloads.random_porosity_3d(shape=shape, seed=4, ell=3.0, nu=0.03, b=2e-4)
        m = np.zeros(shape, np.uint8)
        m[1:3, 5:8, 200:230] = 1             # a block inside the domain
        m[:, 0, :] = 1                       # one wall row (its neighbours y = 1, y = ny - 1)
    else:
        shape = (1, 40, 400)
        w = workloads.random_porosity_2d(nx=400, ny=40, seed=4, ell=4.0, nu=0.04, b=2e-4)
        m = np.zeros(shape, np.uint8)
        m[0, 18:21, 100:103] = 1
    w.mask = m
    st = capi.LBM_F64 if storage == "f64" else capi.LBM_F16_SHIFTED
    s, o = _run_pair(w, 41, storage=st, lagged=lagged, shift=capi.LBM_SHIFT_POROUS)
    s.step(40)
    o.step(40)
    errs = _field_errors(s, o)
    _print(f"solid-free tiles D{D} lagged={lagged} {storage}:", errs)
    if storage == "f64":
        assert max(errs.values()) <= FP64_TOL, errs
    else:
        assert errs["f"] < 1e-4 and errs["rho"] < 1e-4, errs


@pytest.mark.parametrize("storage,lagged", [("f64", False), ("f32", False), ("f32", True),
                                            ("f16", False), ("f16", True), ("bf16", False),
                                            ("bf16", True)])
def test_packed_rows_match_rectangular_tiles(storage, lagged):
    """Runs whose x extent is not a multiple of 64 use packed-row tiles; the tile mapping
    decides only which thread updates which cell, so the result is bitwise that of the
    rectangular tiles (ragged 70 x 13 x 9 with solid blocks, both AA phases).  The 16-bit forms
    (porous shift) read the porosity of their decode through the caches on packed rows and from
    LDS on rectangular tiles (45 % of the lanes of 70-cell rows idle: packed)."""
    w = _solids_3d(shape=(9, 13, 70))
    st = {"f64": capi.LBM_F64, "f32": capi.LBM_F32, "f16": capi.LBM_F16_SHIFTED,
          "bf16": capi.LBM_BF16_SHIFTED}[storage]
    scheme = capi.LBM_SCHEME_LAGGED if lagged else capi.LBM_SCHEME_TWO_PASS
    out = []
    for tiles in (capi.LBM_TILES_AUTO, capi.LBM_TILES_RECTANGULAR):
        s = capi.Solver.from_workload(w, storage=st, scheme=scheme, tiles=tiles,
                                      shift=capi.LBM_SHIFT_POROUS)
        s.step(21)
        f = s.populations(torch.float64).cpu().numpy()
        rho, v = (t.cpu().numpy() for t in s.moments(torch.float64))
        out.append((f, rho, v))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_lagged_restart_takes_a_two_pass_step():
    """After lbm_set_populations the lagged history restarts: the next step is a two-pass step,
    as in the oracle, and the run continues lagged from there."""
    w = _solids_3d(shape=(6, 7, 9))
    s, o = _run_pair(w, 5, lagged=True)
    s.set_populations(s.populations(), step=5)
    o.set_populations(o.populations(), t=5)
    s.step(4)
    o.step(4)
    errs = _field_errors(s, o)
    _print("lagged restart:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    assert s.step_count == 9


def test_lagged_statistics_match_oracle():
    w = workloads.random_porosity_2d(nx=40, ny=30, seed=8, ell=4.0, nu=0.05, b=1e-4)
    s, o = _run_pair(w, 0, lagged=True)
    s.residual()
    o.stats()
    for _ in range(2):
        s.step(25)
        o.step(25)
        g, r = s.residual(), o.stats()
        assert abs(g.mass - r["mass"]) <= 1e-13 * r["mass"]
        assert abs(g.vmax - r["vmax"]) <= 1e-12 * r["vmax"]
        assert abs(g.residual - r["residual"]) <= 1e-10 * r["residual"]


def test_lagged_fp32_tracks_fp64_oracle():
    """FP32 lagged scheme against the FP64 lagged oracle on the random-porosity recipe (32^3,
    100 steps), with the tolerances of the two-pass FP32 case (measured on MI355X: f 2.3e-6,
    rho 2.2e-6, v 1.7e-4..3.2e-4)."""
    w = workloads.random_porosity_3d(shape=(32, 32, 32), seed=0, ell=16.0)
    s, o = _run_pair(w, 100, storage=capi.LBM_F32, lagged=True)
    errs = _field_errors(s, o)
    _print("lagged fp32 vs fp64 oracle:", errs)
    assert errs["f"] < 5e-6 and errs["rho"] < 5e-6
    assert max(errs[k] for k in ("v0", "v1", "v2")) < 7e-4


# --------------------------------------------------------------------------------------------
# Statistics, checkpoints, outputs
# --------------------------------------------------------------------------------------------
def test_residual_statistics_match_oracle():
    w = workloads.random_porosity_2d(nx=40, ny=30, seed=8, ell=4.0, nu=0.05, b=1e-4)
    m = np.zeros(w.shape, np.uint8)
    m[0, 0, :] = m[0, -1, :] = 1
    w.mask = m
    s = capi.Solver.from_workload(w, storage=capi.LBM_F64)
    o = _oracle_for(w)
    g0, r0 = s.residual(), o.stats()
    assert math.isinf(g0.residual) and math.isinf(r0["residual"])
    for _ in range(3):
        s.step(50)
        o.step(50)
        g, r = s.residual(), o.stats()
        assert abs(g.mass - r["mass"]) <= 1e-13 * r["mass"]
        np.testing.assert_allclose([g.momentum[0], g.momentum[1]], r["momentum"][:2],
                                   rtol=1e-11, atol=1e-20)
        assert abs(g.vmax - r["vmax"]) <= 1e-12 * r["vmax"]
        assert abs(g.residual - r["residual"]) <= 1e-10 * r["residual"]
        assert g.nonfinite == 0 and g.step == s.step_count


def test_checkpoint_roundtrip_is_exact():
    """get/set populations (natural layout) resumes bit for bit, from either AA phase."""
    w = workloads.random_porosity_3d(shape=(8, 9, 10), seed=2, ell=2.0, nu=0.03, b=2e-4)
    w.mask = np.zeros(w.shape, np.uint8)
    w.mask[3:5, 3:5, 3:5] = 1
    for storage in (capi.LBM_F64, capi.LBM_F32):
        a = capi.Solver.from_workload(w, storage=storage)
        b = capi.Solver.from_workload(w, storage=storage)
        a.step(7)                                   # odd: swapped AA layout
        b.step(7)
        ck = b.populations()
        b.step(3)
        b.set_populations(ck, step=7)
        assert b.step_count == 7
        a.step(6)
        b.step(6)
        fa, fb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
        assert np.array_equal(fa, fb)


def test_intrinsic_velocity_output():
    w = workloads.random_porosity_2d(nx=20, ny=16, seed=1, ell=3.0, nu=0.05, b=1e-4)
    s = capi.Solver.from_workload(w, storage=capi.LBM_F64)
    s.step(5)
    _, v = s.moments(torch.float64)
    _, u = s.moments(torch.float64, intrinsic=True)
    eps = torch.from_numpy(w.eps).to(v.device)
    torch.testing.assert_close(u * eps, v, rtol=1e-15, atol=0)
    rho32, v32 = s.moments(torch.float32)
    assert rho32.dtype == torch.float32
    torch.testing.assert_close(v32.double(), v, rtol=1e-7, atol=1e-12)


# --------------------------------------------------------------------------------------------
# FP32 storage against the FP64 oracle
# --------------------------------------------------------------------------------------------
def test_d3q27_fp32_tracks_fp64_oracle():
    """FP32 storage and arithmetic against the FP64 oracle on the random-porosity recipe
    (32^3, l = 16, nu = 0.01, b = 1e-6, 100 steps).  Tolerance model: each step rounds every
    population (~0.3) a few times at u = 6e-8, so after n steps f-bar drifts by ~sqrt(n) * 5u
    ~ 3e-6 of its maximum; rho = S/eps sums 27 of them (~1e-5); v is a difference of
    populations divided by rho, ~1e-8 absolute against |v| ~ 1e-5..1e-4 here.  Measured on
    MI355X: f 2.2e-6, rho 2.3e-6, v 1.4e-4..2.8e-4; the bounds below leave a factor ~2."""
    w = workloads.random_porosity_3d(shape=(32, 32, 32), seed=0, ell=16.0)
    s, o = _run_pair(w, 100, storage=capi.LBM_F32)
    errs = _field_errors(s, o)
    _print("d3q27 fp32 vs fp64 oracle:", errs)
    assert errs["f"] < 5e-6 and errs["rho"] < 5e-6
    assert max(errs[k] for k in ("v0", "v1", "v2")) < 6e-4


# --------------------------------------------------------------------------------------------
# Shifted 16-bit population storage against the FP64 oracle
# --------------------------------------------------------------------------------------------
def _l2_linf(a, b):
    d = (a - b).ravel()
    r = b.ravel()
    return float(np.linalg.norm(d) / np.linalg.norm(r)), float(np.abs(d).max() / np.abs(r).max())


_SHIFTED = {"f16": capi.LBM_F16_SHIFTED, "bf16": capi.LBM_BF16_SHIFTED}
_SHIFTS = {"weights": capi.LBM_SHIFT_WEIGHTS, "porous": capi.LBM_SHIFT_POROUS}


# Bounds are 2-3x the errors measured on MI355X (v L2 / v Linf / f / mass drift):
#   f16 porous  1.9e-3 / 2.3e-3 / 1.3e-5 / 5.7e-7     bf16 porous  1.5e-2 / 1.6e-2 / 1.1e-4 / 2.9e-7
#   f16 weights 4.8e-2 / 3.5e-2 / 6.0e-4 / 6.9e-5     bf16 weights 0.38   / 0.29   / 4.7e-3 / 2.3e-4
# (FP32 storage: v 1.6e-4..4e-4).  Model: a stored deviation d carries a relative rounding
# error of 2^-11 (FP16) or 2^-8 (BF16).  With the porous shift d is the flow's own deviation
# from eps rho0 w_i, ~1e-3 of f here, so FP16 costs about as much as FP32 arithmetic; with the
# weight shift d includes (eps - 1) rho0 w_i, up to 0.7 w_i at eps = 0.3, and the velocity error
# grows ~25-fold.
_SHIFT_BOUNDS = {("f16", "porous"): (4e-3, 5e-3, 3e-5, 2e-6),
                 ("bf16", "porous"): (3e-2, 3.5e-2, 2.5e-4, 1e-6),
                 ("f16", "weights"): (0.1, 0.08, 1.3e-3, 1.5e-4),
                 ("bf16", "weights"): (0.8, 0.6, 1e-2, 5e-4)}


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("shift", ["weights", "porous"])
def test_shifted_storage_velocity_error(fmt, shift):
    """Populations stored as 16-bit shifted deviations, FP32 collision, FP64 statistics, against
    the FP64 oracle on the random-porosity recipe (32^3, l = 16, nu = 0.01, b = 1e-6, 100
    steps): the L2 and Linf velocity errors and the mass drift within the stated bounds."""
    w = workloads.random_porosity_3d(shape=(32, 32, 32), seed=0, ell=16.0)
    s, o = _run_pair(w, 100, storage=_SHIFTED[fmt], shift=_SHIFTS[shift])
    _, v_gpu = (t.cpu().numpy() for t in s.moments(torch.float64))
    _, v_ref, _ = o.moments()
    l2, linf = _l2_linf(v_gpu, v_ref)
    mass_gpu, mass_ref = s.residual().mass, o.stats()["mass"]
    drift = abs(mass_gpu - mass_ref) / mass_ref
    errs = _field_errors(s, o)
    print(f"shifted {fmt}/{shift}: v L2 {l2:.3e} Linf {linf:.3e} mass {drift:.3e}", flush=True)
    _print(f"shifted {fmt}/{shift} fields:", errs)
    b_l2, b_linf, b_f, b_m = _SHIFT_BOUNDS[(fmt, shift)]
    assert l2 < b_l2 and linf < b_linf and errs["f"] < b_f and drift < b_m


@pytest.mark.parametrize("lagged", [False, True])
def test_porous_shift_with_solids(lagged):
    """FP16 storage with the porous shift next to solid cells inside a varying porosity field,
    both schemes: a value produced by a bounce-back is shifted with the porosity of the cell
    that bounced it.  A reader that took the upstream (solid) cell's porosity instead would be
    off by (eps_a - eps_b) w_i ~ 1e-2 of f here, far above the bound."""
    w = _solids_3d(shape=(10, 12, 40))
    w.eta_eff = float("nan")
    s, o = _run_pair(w, 40, storage=capi.LBM_F16_SHIFTED, lagged=lagged,
                     shift=capi.LBM_SHIFT_POROUS)
    errs = _field_errors(s, o)
    _print(f"f16 porous solids lagged={lagged}:", errs)
    assert errs["f"] < 1e-4 and errs["rho"] < 1e-4
    assert max(errs[k] for k in ("v0", "v1", "v2")) < 2e-2


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_shifted_checkpoint_is_exact_through_fp64(fmt):
    """A 16-bit state exported in FP64 (exact decode) and imported again (exact re-encode: the
    scales are powers of two) continues bit for bit, from either AA phase."""
    w = _solids_3d(shape=(8, 9, 10))
    for steps in (6, 7):
        a = capi.Solver.from_workload(w, storage=_SHIFTED[fmt], shift=capi.LBM_SHIFT_POROUS)
        b = capi.Solver.from_workload(w, storage=_SHIFTED[fmt], shift=capi.LBM_SHIFT_POROUS)
        a.step(steps)
        b.step(steps)
        ck = b.populations(torch.float64)
        b.step(3)
        b.set_populations(ck, step=steps)
        a.step(5)
        b.step(5)
        fa = a.populations(torch.float64).cpu().numpy()
        fb = b.populations(torch.float64).cpu().numpy()
        assert np.array_equal(fa, fb)


# --------------------------------------------------------------------------------------------
# The tile paths of the full-size runs: 256- and 128-wide rectangular row tiles (the 256^3
# headline and the 768-wide duct use 256 x 1 tiles), several y blocks with a partial one, the
# XCD split of the tile order, the z-marching velocity correction over several chunks, the
# rotated stores of the swapped AA phase, and the 258-wide LDS porosity halo of the 16-bit
# forms.
# --------------------------------------------------------------------------------------------
def _wide_case(shape, solids, nu=0.04, b=3e-4, seed=21):
    w = workloads.random_porosity_3d(shape=shape, seed=seed, ell=3.0, nu=nu, b=b)
    if solids:
        nz, ny, nx = shape
        m = np.zeros(shape, np.uint8)
        m[2:5, 30:37, 100:140] = 1          # a block inside
        m[:, 0, :] = 1                      # one wall row (periodic neighbours y = 1, ny - 1)
        m[5:7, :, nx - 3:nx] = 1            # a slab at the x seam of the last tile
        w.mask = m
    return w


@pytest.mark.parametrize("shape", [(12, 72, 256), (10, 20, 128)])
@pytest.mark.parametrize("solids", [False, True])
@pytest.mark.parametrize("lagged", [False, True])
def test_full_width_tiles_fp64(shape, solids, lagged):
    """FP64 on the tile shapes of the full-size runs (x extents 256 and 128, rectangular tiles),
    both schemes, with and without solid cells, against the oracle to 1e-12 after 7 steps (the
    swapped AA layout) and after 12."""
    w = _wide_case(shape, solids)
    s, o = _run_pair(w, 7, lagged=lagged)
    errs = _field_errors(s, o)
    _print(f"wide {shape} solids={solids} lagged={lagged} t=7:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    s.step(5)
    o.step(5)
    errs = _field_errors(s, o)
    _print(f"wide {shape} solids={solids} lagged={lagged} t=12:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


# Bounds for 9 steps at (12, 72, 256), b = 3e-4 (v up to ~3e-3): about 2x the errors measured on
# MI355X (f / rho / v: FP32 1.1e-6 / 7.5e-7 / 1.1e-5, FP16 4.0e-5 / 3.5e-5 / 7.0e-4, BF16
# 2.8e-4 / 3.0e-4 / 5.5e-3), printed by the test.  FP32: every population is rounded (u = 6e-8) a few times per step;
# 16-bit forms: each stored deviation from the porous shift carries a relative error of 2^-11
# (FP16) or 2^-8 (BF16) of a deviation ~1e-3 of f here.
_WIDE_BOUNDS = {"f32": dict(f=2.5e-6, rho=2e-6, v=2.5e-5),
                "f16": dict(f=8e-5, rho=8e-5, v=1.5e-3),
                "bf16": dict(f=6e-4, rho=6e-4, v=1.2e-2)}


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("solids", [False, True])
def test_full_width_tiles_reduced_precision(fmt, solids):
    """FP32 and shifted FP16/BF16 storage (porous shift) on the 256-wide tiles (the 16-bit
    forms stage a 258-wide porosity halo in LDS) against the FP64 oracle, velocity included."""
    w = _wide_case((12, 72, 256), solids)
    st = {"f32": capi.LBM_F32, "f16": capi.LBM_F16_SHIFTED, "bf16": capi.LBM_BF16_SHIFTED}[fmt]
    s, o = _run_pair(w, 9, storage=st, shift=capi.LBM_SHIFT_POROUS)
    errs = _field_errors(s, o)
    _print(f"wide {fmt} solids={solids}:", errs)
    bd = _WIDE_BOUNDS[fmt]
    assert errs["f"] < bd["f"] and errs["rho"] < bd["rho"], errs
    assert max(errs[k] for k in ("v0", "v1", "v2")) < bd["v"], errs


def _sampled_cells(shape, rng, k=3000):
    """Random cells plus the edges the tile order and the z-march produce: x = 0, 63, 64, 255
    (wave and tile edges), y at the 64-row block edges, z at the 4-plane block edges and at the
    16-plane chunk edges of the velocity correction."""
    nz, ny, nx = shape
    xs = rng.integers(0, nx, k)
    ys = rng.integers(0, ny, k)
    zs = rng.integers(0, nz, k)
    ex = np.array([0, 1, 62, 63, 64, 65, 127, 128, 191, 192, nx - 1])
    ey = np.array([0, 1, 63, 64, 127, 128, ny - 1])
    ez = np.array([0, 3, 4, 15, 16, 17, 31, 32, nz - 1])
    gx, gy, gz = np.meshgrid(ex, ey, ez, indexing="ij")
    xs = np.concatenate([xs, gx.ravel()])
    ys = np.concatenate([ys, gy.ravel()])
    zs = np.concatenate([zs, gz.ravel()])
    return np.unique(xs + nx * (ys + ny * zs))


@pytest.mark.parametrize("fmt,steps", [("f32", 3), ("f32", 4), ("f16", 3)])
def test_headline_box_sampled_cells(fmt, steps):
    """The 256^3 random-porosity box (seed 0, l = 16, phi in (0.3, 1), nu = 0.01, b = 1e-6) in
    the launch configuration of the benchmark: after `steps` steps (odd: the swapped AA layout
    is read next) the state is exported, the oracle evaluates the post-collision populations of
    about 3,000 cells from that state in FP64, and one more GPU step must have streamed exactly
    those values (within the rounding of one step of the storage format) to x + c_i."""
    rng = np.random.default_rng(5)
    w = workloads.random_porosity_3d(n=256, seed=0, ell=16.0)
    st = capi.LBM_F32 if fmt == "f32" else capi.LBM_F16_SHIFTED
    s = capi.Solver.from_workload(w, storage=st, shift=capi.LBM_SHIFT_POROUS)
    s.step(steps)
    f0 = s.populations(torch.float64).cpu().numpy()
    s.step(1)
    f1 = s.populations(torch.float64).cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    o = _oracle_for(w)
    o.set_populations(f0, t=steps)
    del f0
    cells = _sampled_cells(w.shape, rng)
    ref = o.post_collision(cells)                       # [ncells, Q], FP64 from the same state
    del o
    c, _ = oracle.lattice(3)
    nz, ny, nx = w.shape
    x, y, z = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    got = np.empty_like(ref)
    f1 = f1.reshape(27, -1)
    for i in range(27):
        d = (x + c[i, 0]) % nx + nx * (((y + c[i, 1]) % ny) + ny * ((z + c[i, 2]) % nz))
        got[:, i] = f1[i, d]
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"headline {fmt} sampled step {steps}->{steps + 1}: {len(cells)} cells, max rel err "
          f"{err:.2e}", flush=True)
    # one step of FP32 arithmetic on populations ~0.3: a few ulp (6e-8); FP16 storage: the
    # stored deviation (|f - eps rho0 w_i| ~ 1e-5 w_i here) scaled to ~4096 carries 2^-11
    assert err < (2e-6 if fmt == "f32" else 2e-5), err


# --------------------------------------------------------------------------------------------
# Small periodic boxes whose neighbour stencils wrap onto themselves
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(7, 16, 64), (3, 8, 32), (1, 8, 32), (2, 24, 96),
                                   (21, 16, 32)])
def test_small_periodic_boxes_fp64(shape):
    """One, two and three planes (the z neighbours are the plane itself or the other one),
    rows of one 32- or 64-cell wave, several tile blocks along z, with every option of the
    forcing on (RT != 1/3, Phi^eta, nu_eff = nu_ref / eps): bitwise to the oracle after 5
    steps (swapped AA layout next) and after 8."""
    w = workloads.random_porosity_3d(shape=shape, seed=17, ell=2.5, nu=0.03, b=2e-4)
    w.RT = 0.36
    w.eta_eff = 0.02
    w.nu_eff_pow = -1
    s, o = _run_pair(w, 5)
    errs = _field_errors(s, o)
    _print(f"small box {shape} t=5:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    s.step(3)
    o.step(3)
    errs = _field_errors(s, o)
    _print(f"small box {shape} t=8:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


def test_analytic_derivatives_on_a_tile_multiple_box():
    """Analytic porosity derivatives (Sec. 3.5) on a box of whole 32-cell rows and 8-row tile
    blocks, against the oracle given the same derivatives."""
    w = workloads.sine_porosity(D=3, shape=(8, 16, 32))
    s = capi.Solver.from_workload(w, storage=capi.LBM_F64)
    o = _oracle_for(w, grad_eps=w.grad_eps, hess_eps=w.hess_eps)
    s.step(6)
    o.step(6)
    torch.cuda.synchronize()
    errs = _field_errors(s, o)
    _print("analytic box:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


# --------------------------------------------------------------------------------------------
# Velocity correction inside the collision pass (LBM_PASSES_AUTO)
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("shape,opts", [((12, 8, 64), False), ((40, 16, 128), True),
                                        ((3, 8, 64), True), ((17, 8, 192), False)])
def test_fused_correction_pass_fp64(shape, opts):
    """Shapes that take the fused correction-collision kernel (x a multiple of 64, y of 8, no
    solids): one to three 64-cell tiles along x, y tiles whose ring wraps onto the tile itself,
    z-chunks of 32 planes with a partial last one and a three-plane box, with and without every
    forcing option (RT != 1/3, Phi^eta, nu_eff = nu_ref / eps): bitwise (1e-12) to the oracle
    after 5 steps and after 8; the timed step reports no separate correction kernel."""
    w = workloads.random_porosity_3d(shape=shape, seed=23, ell=3.0, nu=0.03, b=2e-4)
    if opts:
        w.RT = 0.36
        w.eta_eff = 0.02
        w.nu_eff_pow = -1
    s = capi.Solver.from_workload(w, storage=capi.LBM_F64, passes=capi.LBM_PASSES_FUSED)
    o = _oracle_for(w)
    s.step(5)
    o.step(5)
    errs = _field_errors(s, o)
    _print(f"fused {shape} opts={opts} t=5:", errs)
    assert max(errs.values()) <= FP64_TOL, errs
    ms = s.step_timed(3)
    o.step(3)
    assert ms[1] == 0.0 and ms[2] > 0.0, ms
    errs = _field_errors(s, o)
    _print(f"fused {shape} opts={opts} t=8:", errs)
    assert max(errs.values()) <= FP64_TOL, errs


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_fused_and_separate_passes_are_bitwise_equal(storage):
    """FP32 and shifted 16-bit storage (porous shift): the fused correction-collision kernel
    and the separate correction pass evaluate the same expressions, so 7 steps (both AA phases)
    give identical populations and moments (z-chunks of 8 planes, 3 of them in the 20-plane
    box)."""
    w = workloads.random_porosity_3d(shape=(20, 16, 128), seed=3, ell=4.0)
    st = {"f32": capi.LBM_F32, "f16": capi.LBM_F16_SHIFTED, "bf16": capi.LBM_BF16_SHIFTED}[storage]
    kw = dict(storage=st, shift=capi.LBM_SHIFT_POROUS)
    a = capi.Solver.from_workload(w, passes=capi.LBM_PASSES_FUSED, **kw)
    b = capi.Solver.from_workload(w, passes=capi.LBM_PASSES_SEPARATE, **kw)
    ta, tb = a.step_timed(7), b.step_timed(7)
    assert ta[1] == 0.0 and tb[1] > 0.0, (ta, tb)
    assert torch.equal(a.populations(torch.float64), b.populations(torch.float64))
    for x, y in zip(a.moments(torch.float64), b.moments(torch.float64)):
        assert torch.equal(x, y)
