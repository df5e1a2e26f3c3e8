"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point
that include/lbm.h declares, numbers the lattices as the paper's wall example does, sizes its
workspace, and rejects invalid runs before touching the device."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2606_29619_amd import capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "lbm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"LBM_API\s+[\w\s\*]+?\b(lbm_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 12, names
    lib = capi.load()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lbm.h but not exported"


def test_no_undeclared_exports():
    """The shared library exports the C ABI and nothing else of its own (hidden visibility)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    ours = sorted({l.split()[-1] for l in out.splitlines() if l.split()[-1].startswith("lbm_")})
    assert ours == _declared()


@pytest.mark.parametrize("lattice,D", [(capi.LBM_D2Q9, 2), (capi.LBM_D3Q27, 3)])
def test_lattice_numbering_matches_oracle(lattice, D):
    """Both sides define the lattice tables independently; they must agree on the numbering,
    which fixes the summation order of the moments."""
    c_lib, opp_lib = capi.lbm_lattice_info(lattice)
    c_orc, opp_orc = oracle.lattice(D)
    np.testing.assert_array_equal(c_lib, c_orc)
    np.testing.assert_array_equal(opp_lib, opp_orc)


def _params(lattice=capi.LBM_D3Q27, storage=capi.LBM_F32, shape=(4, 5, 6), mask=None, **kw):
    eps = np.full(shape, 0.5)
    base = dict(kappa=np.full(shape, 0.1), forch=np.full(shape, 1.0))
    base.update({k: kw.pop(k) for k in list(kw) if k in ("kappa", "forch", "eps")})
    if "eps" in base:
        eps = base.pop("eps")
    return capi.make_params(lattice, storage, eps, base["kappa"], base["forch"], mask, **kw)


def test_footprint_sizes():
    p, _ = _params(shape=(4, 5, 6))
    N = 120
    fp = capi.lbm_footprint(p)
    # populations + 3 static + two 4-value moment records + D-component residual snapshot +
    # reduction scratch, each region 256-byte aligned
    assert fp >= (27 + 3 + 8 + 3) * N * 4
    assert fp < (27 + 3 + 8 + 3) * N * 4 + 20 * 256 + 1024 * 8 * 8 + 64
    p64, _ = _params(storage=capi.LBM_F64)
    assert capi.lbm_footprint(p64) > fp
    pm, _ = _params(mask=np.zeros((4, 5, 6), np.uint8))
    assert capi.lbm_footprint(pm) > fp
    # the lagged scheme double-buffers both records
    pl, _ = _params(scheme=capi.LBM_SCHEME_LAGGED)
    assert capi.lbm_footprint(pl) - fp >= 8 * N * 4
    assert capi.lbm_footprint(pl) - fp < 8 * N * 4 + 2 * 256
    # 16-bit populations, FP32 static fields and records
    for st in (capi.LBM_F16_SHIFTED, capi.LBM_BF16_SHIFTED):
        ph, _ = _params(storage=st)
        assert fp - capi.lbm_footprint(ph) >= 27 * N * 2 - 256
        assert fp - capi.lbm_footprint(ph) <= 27 * N * 2 + 256
    # the population region also stages four FP64 input arrays at creation
    p2, _ = _params(lattice=capi.LBM_D2Q9, storage=capi.LBM_F16_SHIFTED, shape=(1, 8, 8))
    assert capi.lbm_footprint(p2) >= 4 * 64 * 8 + (3 + 8 + 2) * 64 * 4


@pytest.mark.parametrize("mutate,code", [
    (dict(lattice=15), capi.LBM_ERR_INVALID_ARG),
    (dict(storage=9), capi.LBM_ERR_UNSUPPORTED),
    (dict(nx=0), capi.LBM_ERR_INVALID_ARG),
    (dict(scheme=2), capi.LBM_ERR_INVALID_ARG),
    (dict(shift=5), capi.LBM_ERR_INVALID_ARG),
    (dict(storage=4), capi.LBM_ERR_UNSUPPORTED),
])
def test_footprint_rejects_bad_shape(mutate, code):
    p, _ = _params()
    for k, v in mutate.items():
        setattr(p, k, v)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(p)
    assert ei.value.code == code


def test_d2q9_requires_nz_1():
    p, _ = _params(lattice=capi.LBM_D2Q9, shape=(2, 4, 4))
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(p)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG


@pytest.mark.parametrize("case", [
    "eps_zero", "eps_above_one", "eps_nan", "kappa_zero", "forch_negative", "rho0", "RT",
    "nu_eff", "pow", "eta", "null_ws", "small_ws", "misaligned_ws", "all_solid", "mask_value",
])
def test_create_rejects_invalid_runs_before_device_work(case):
    """lbm_create validates everything on the host; these calls never reach the GPU (the
    workspace pointers below are fake and are never dereferenced)."""
    shape = (4, 5, 6)
    eps = np.full(shape, 0.5)
    kappa = np.full(shape, 0.1)
    forch = np.full(shape, 1.0)
    mask = None
    kw = {}
    if case == "eps_zero":
        eps[1, 2, 3] = 0.0
    elif case == "eps_above_one":
        eps[0, 0, 0] = 1.5
    elif case == "eps_nan":
        eps[0, 0, 1] = math.nan
    elif case == "kappa_zero":
        kappa[3, 1, 1] = 0.0
    elif case == "forch_negative":
        forch[2, 2, 2] = -1.0
    elif case == "rho0":
        kw["rho0"] = 0.0
    elif case == "RT":
        kw["RT"] = -0.1
    elif case == "nu_eff":
        kw["nu_eff_ref"] = 0.0
    elif case == "pow":
        kw["nu_eff_pow"] = 2
    elif case == "eta":
        kw["eta_eff"] = -1.0
    elif case == "all_solid":
        mask = np.ones(shape, np.uint8)
    elif case == "mask_value":
        mask = np.zeros(shape, np.uint8)
        mask[0, 0, 0] = 7
    p, keep = capi.make_params(capi.LBM_D3Q27, capi.LBM_F32, eps, kappa, forch, mask, **kw)
    need = capi.lbm_footprint(p)
    ws, nbytes = 1 << 20, need
    if case == "null_ws":
        ws = 0
    elif case == "small_ws":
        nbytes = need - 1
    elif case == "misaligned_ws":
        ws = (1 << 20) + 4
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_create(p, ws, nbytes, 0)
    expect = capi.LBM_ERR_WORKSPACE if case in ("small_ws", "misaligned_ws") else \
        capi.LBM_ERR_INVALID_ARG
    assert ei.value.code == expect, capi.lbm_last_error()
    assert capi.lbm_last_error()


def test_solid_cells_may_hold_any_permeability():
    """kappa and C_F are read on fluid cells only; eps must be valid everywhere (it enters the
    porosity derivatives).  A solid cell with kappa = 0 is accepted up to the workspace check."""
    shape = (4, 5, 6)
    kappa = np.full(shape, 0.1)
    kappa[0, 0, 0] = 0.0
    mask = np.zeros(shape, np.uint8)
    mask[0, 0, 0] = 1
    p, keep = capi.make_params(capi.LBM_D3Q27, capi.LBM_F32, np.full(shape, 0.5), kappa,
                               np.ones(shape), mask)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_create(p, 1 << 20, 10, 0)
    assert ei.value.code == capi.LBM_ERR_WORKSPACE


def test_null_handle_calls_fail_cleanly():
    lib = capi.load()
    assert lib.lbm_step(None, 1) == capi.LBM_ERR_INVALID_ARG
    assert lib.lbm_residual(None, None) == capi.LBM_ERR_INVALID_ARG
    assert lib.lbm_destroy(None) == capi.LBM_OK


# --------------------------------------------------------------------------------------------
# Request server: host-side validation and bookkeeping (no device work before progress)
# --------------------------------------------------------------------------------------------
_FAKE_POOL = 1 << 40          # 256-byte aligned, never dereferenced by these calls


def test_server_rejects_bad_configuration():
    for args, code in [((_FAKE_POOL, 1 << 30, 99, 0), capi.LBM_ERR_INVALID_ARG),   # odd round
                       ((_FAKE_POOL, 1 << 30, 0, 0), capi.LBM_ERR_INVALID_ARG),
                       ((_FAKE_POOL, 1 << 30, 100, -1), capi.LBM_ERR_INVALID_ARG),
                       ((_FAKE_POOL, 1 << 10, 100, 0), capi.LBM_ERR_WORKSPACE),    # tiny pool
                       ((_FAKE_POOL + 8, 1 << 30, 100, 0), capi.LBM_ERR_WORKSPACE)]:
        with pytest.raises(capi.LbmError) as ei:
            capi.lbm_server_create(*args, 0)
        assert ei.value.code == code, args


def test_server_submit_copies_and_queues():
    s = capi.lbm_server_create(_FAKE_POOL, 1 << 30, 100, 0, 0)
    try:
        p, keep = _params(shape=(4, 5, 6))
        rid = capi.lbm_server_submit(s, p, 1e-7, 1000)
        keep[0][:] = 7.0                           # the server holds its own copy
        p2, keep2 = _params(lattice=capi.LBM_D2Q9, shape=(1, 8, 8))
        rid2 = capi.lbm_server_submit(s, p2, 1e-6, 200)
        assert (rid, rid2) == (0, 1)
        info = capi.lbm_server_info(s, rid)
        assert info.state == capi.LBM_REQ_QUEUED and info.cells == 120
        assert info.workspace_bytes == capi.lbm_footprint(_params(shape=(4, 5, 6))[0])
        assert info.t_admit == -1 and info.t_done == -1 and info.steps == 0
        st = capi.lbm_server_get_stats(s)
        assert (st.submitted, st.queued, st.active, st.pool_used) == (2, 2, 0, 0)
        with pytest.raises(capi.LbmError) as ei:          # not finished
            capi.lbm_server_release(s, rid)
        assert ei.value.code == capi.LBM_ERR_STATE
        with pytest.raises(capi.LbmError) as ei:          # holds no state yet
            capi.lbm_server_solver(s, rid)
        assert ei.value.code == capi.LBM_ERR_STATE
        for bad in [dict(tol=0.0), dict(max_steps=50), dict(floor_checks=-1)]:
            kw = dict(tol=1e-7, max_steps=1000, floor_checks=0)
            kw.update(bad)
            with pytest.raises(capi.LbmError) as ei:
                capi.lbm_server_submit(s, p, kw["tol"], kw["max_steps"], kw["floor_checks"])
            assert ei.value.code == capi.LBM_ERR_INVALID_ARG
        big, keep3 = _params(shape=(96, 96, 96))
        with pytest.raises(capi.LbmError) as ei:          # can never fit a 64 MiB pool
            s2 = capi.lbm_server_create(_FAKE_POOL, 64 << 20, 100, 0, 0)
            try:
                capi.lbm_server_submit(s2, big, 1e-7, 1000)
            finally:
                capi.lbm_server_destroy(s2)
        assert ei.value.code == capi.LBM_ERR_WORKSPACE
    finally:
        capi.lbm_server_destroy(s)


# --------------------------------------------------------------------------------------------
# Wet-node boundaries: host-side validation
# --------------------------------------------------------------------------------------------
def _bc_params(**over):
    from paper_2606_29619_amd import workloads
    w = workloads.couette_gravity_2d(H=8)
    kw = dict(bc_type=w.bc_type, bc_normal=w.bc_normal, bc_velocity=w.bc_velocity)
    kw.update(over)
    return capi.make_params(capi.LBM_D2Q9, capi.LBM_F64, w.eps, w.kappa, w.forch, w.mask,
                            rho_init=w.rho_init, **kw), w


def test_boundary_footprint_and_validation():
    (p, keep), w = _bc_params()
    (p0, keep0), _ = _bc_params(bc_type=None)
    nb = int((w.bc_type > 0).sum())
    assert capi.lbm_footprint(p) - capi.lbm_footprint(p0) >= nb * (4 + 4 + 32)
    # lagged scheme: accepted with wet-node boundaries, double-buffered records cost more
    p.scheme = capi.LBM_SCHEME_LAGGED
    assert capi.lbm_footprint(p) > capi.lbm_footprint(p0)
    # Picard iterations stay two-pass only
    (p5, keep5), _ = _bc_params(picard_iters=2)
    p5.scheme = capi.LBM_SCHEME_LAGGED
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(p5)
    assert ei.value.code == capi.LBM_ERR_UNSUPPORTED
    # a boundary node whose outward neighbour is fluid
    bct = w.bc_type.copy()
    bct[0, 3, 1] = 1
    (p2, keep2), _ = _bc_params(bc_type=bct)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_create(p2, 1 << 40, 1 << 30, 0)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG and "outward" in str(ei.value)
    # a bad normal code and a bad scheme
    bcn = w.bc_normal.copy()
    bcn[0, 1, 0] = 4                   # -z on a D2Q9 grid
    (p3, keep3), _ = _bc_params(bc_normal=bcn)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(p3)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG
    (p4, keep4), _ = _bc_params(bc_scheme=7)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(p4)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG


def _box_params(w, **over):
    kw = dict(bc_type=w.bc_type, bc_normal=w.bc_normal, bc_velocity=w.bc_velocity,
              bc_density=w.bc_density)
    kw.update(over)
    return capi.make_params(capi.LBM_D2Q9, capi.LBM_F64, w.eps, w.kappa, w.forch, w.mask, **kw)


def test_edge_and_corner_node_validation():
    """Edge and corner nodes (Sec. 3.4.1): velocity nodes with every listed outward neighbour
    solid and two bulk fluid cells along the inward diagonal; codes are LBM_NORMAL_* or
    LBM_NORMAL_AXES."""
    from paper_2606_29619_amd import workloads
    w = workloads.wet_box(2, (8, 6, 1), faces={"x-": "inlet", "x+": "pressure"})
    assert w.bc_normal[0, 1, 1] == capi.LBM_NORMAL_AXES(-1, -1)
    p, keep = _box_params(w)
    assert capi.lbm_footprint(p) > 0

    def rejects(bct=None, bcn=None, what=""):
        pp, kk = _box_params(w, bc_type=w.bc_type if bct is None else bct,
                             bc_normal=w.bc_normal if bcn is None else bcn)
        with pytest.raises(capi.LbmError) as ei:
            capi.lbm_footprint(pp)
        assert ei.value.code == capi.LBM_ERR_INVALID_ARG and what in str(ei.value), str(ei.value)

    bct = w.bc_type.copy()
    bct[0, 1, -2] = capi.LBM_NODE_PRESSURE                # a corner as a pressure node
    rejects(bct=bct, what="velocity node")
    bcn = w.bc_normal.copy()
    bcn[0, 1, 3] = capi.LBM_NORMAL_AXES(-1, -1)           # a wall node claiming a -x face
    rejects(bcn=bcn, what="outward")
    bcn = w.bc_normal.copy()
    bcn[0, 1, 1] = capi.LBM_NORMAL_AXES(-1, -1, 1)        # a z normal on a D2Q9 grid
    rejects(bcn=bcn)
    bcn = w.bc_normal.copy()
    bcn[0, 1, 1] = 64 + 3                                 # not a sign code
    rejects(bcn=bcn)
    small = workloads.wet_box(2, (8, 2, 1))               # the diagonal runs into the far wall
    pp, kk = _box_params(small)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(pp)
    assert "diagonal" in str(ei.value) or "inward" in str(ei.value), str(ei.value)


def test_server_queues_boundary_runs():
    """Runs with wet-node boundaries are accepted (served on their own launches); a geometry
    the solver would refuse is refused at submission."""
    (p, keep), w = _bc_params()
    s = capi.lbm_server_create(_FAKE_POOL, 1 << 30, 100, 0, 0)
    try:
        rid = capi.lbm_server_submit(s, p, 1e-7, 1000)
        assert capi.lbm_server_info(s, rid).state == capi.LBM_REQ_QUEUED
        bcn = w.bc_normal.copy()
        bcn[0, 1, 0] = 4                   # -z on a D2Q9 grid
        (p3, keep3), _ = _bc_params(bc_normal=bcn)
        with pytest.raises(capi.LbmError) as ei:
            capi.lbm_server_submit(s, p3, 1e-7, 1000)
        assert ei.value.code == capi.LBM_ERR_INVALID_ARG
    finally:
        capi.lbm_server_destroy(s)


def test_picard_validation_and_footprint():
    p, _k = _params(shape=(4, 5, 6))
    base = capi.lbm_footprint(p)
    p.picard_iters, p.picard_omega = 3, 1.0
    assert capi.lbm_footprint(p) - base >= 2 * 4 * 120 * 4          # (rho, v_0) + scratch
    for iters, omega, scheme, code in [(65, 1.0, 0, capi.LBM_ERR_INVALID_ARG),
                                       (2, 0.0, 0, capi.LBM_ERR_INVALID_ARG),
                                       (2, 1.5, 0, capi.LBM_ERR_INVALID_ARG),
                                       (2, 1.0, capi.LBM_SCHEME_LAGGED, capi.LBM_ERR_UNSUPPORTED)]:
        q, _kk = _params(shape=(4, 5, 6))
        q.picard_iters, q.picard_omega, q.scheme = iters, omega, scheme
        with pytest.raises(capi.LbmError) as ei:
            capi.lbm_footprint(q)
        assert ei.value.code == code, (iters, omega, scheme)


def test_analytic_derivative_validation_and_footprint():
    """grad_eps and hess_eps go together, add D + D(D+1)/2 value planes to the workspace, must
    be finite on fluid cells (solid cells are never read), and the server queues such runs."""
    shape = (4, 5, 6)
    N = 120
    p, _k = _params(shape=shape)
    base = capi.lbm_footprint(p)
    g, h = np.zeros((3,) + shape), np.zeros((6,) + shape)
    q, _kq = _params(shape=shape, grad_eps=g, hess_eps=h)
    # nine planes of N values more; the analytic run drops the flat-tile flags (256 B here)
    assert capi.lbm_footprint(q) - base >= 9 * N * 4 - 256
    r, _kr = _params(shape=shape, grad_eps=g)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_footprint(r)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG
    mask = np.zeros(shape, np.uint8)
    mask[0, 0, 0] = 1
    for which, idx, expect in [("grad", (1, 2, 3, 4), "grad_eps"),
                               ("hess", (5, 1, 1, 1), "hess_eps"),
                               ("grad", (2, 0, 0, 0), "dev_workspace")]:   # a solid cell
        gg, hh = g.copy(), h.copy()
        (gg if which == "grad" else hh)[idx] = math.nan
        s, _ks = _params(shape=shape, mask=mask, grad_eps=gg, hess_eps=hh)
        need = capi.lbm_footprint(s)
        with pytest.raises(capi.LbmError) as ei:
            capi.lbm_create(s, 0, need, 0)         # null workspace: fails after the field checks
        assert ei.value.code == capi.LBM_ERR_INVALID_ARG
        assert expect in capi.lbm_last_error(), capi.lbm_last_error()
    srv = capi.lbm_server_create(_FAKE_POOL, 1 << 30, 100, 0, 0)
    try:
        rid = capi.lbm_server_submit(srv, q, 1e-7, 1000)
        assert capi.lbm_server_info(srv, rid).state == capi.LBM_REQ_QUEUED
    finally:
        capi.lbm_server_destroy(srv)


def test_stats_noalloc_rejects_a_null_handle():
    """The allocation-free statistics entry point validates its handle before any device work."""
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_stats_noalloc(None, 0)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG
