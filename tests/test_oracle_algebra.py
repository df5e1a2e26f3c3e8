"""Pins of the oracle's algebra against what the paper and the mathematics fix.

Each test names the passage it checks.  None re-types the oracle's formula: the expected values
are exact rationals, closed-form moment identities, substitution into the defining equation,
or an independent spectral evaluation of a differential operator.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_d2q9_numbering_matches_wall_example():
    """Sec. 3.4.1: the wall-density example fixes tangential {0,1,3}, P+ = {4,7,8} at the
    bottom wall and {2,5,6} at the top wall."""
    c, opp = oracle.lattice(2)
    sets = {r[0]: sorted(int(x) for x in r[1:]) for r in _read_golden("d2q9_wall_sets.txt")}
    assert sorted(np.where(c[:, 1] == 0)[0].tolist()) == sets["tangential"]
    assert sorted(np.where(c[:, 1] == -1)[0].tolist()) == sets["outgoing_bottom"]
    assert sorted(np.where(c[:, 1] == 1)[0].tolist()) == sets["outgoing_top"]
    assert c[1].tolist()[:2] == [1, 0] and c[3].tolist()[:2] == [-1, 0]
    for i in range(9):
        assert (c[opp[i]] == -c[i]).all()


@pytest.mark.parametrize("D", [2, 3])
def test_lattice_is_full_tensor_product(D):
    """Sec. 3.1: D(n)Q(3^n) holds every velocity with components in {-1, 0, 1}."""
    c, opp = oracle.lattice(D)
    Q = 3 ** D
    assert c.shape == (Q, 3)
    got = sorted(tuple(r[:D]) for r in c)
    assert got == sorted(itertools.product((-1, 0, 1), repeat=D))
    assert (c[0] == 0).all()
    for i in range(Q):
        assert (c[opp[i]] == -c[i]).all()


def test_weights_are_textbook_values():
    """Appendix C, eq. (eq_weights) at RT = 1/3 gives the textbook weights."""
    for lat, c2, num, den in _read_golden("lattice_weights.txt"):
        D = 2 if lat == "D2Q9" else 3
        c, _ = oracle.lattice(D)
        w = oracle.weights(D, 1.0 / 3.0)
        sel = (c[:, :D] ** 2).sum(axis=1) == int(c2)
        assert sel.any()
        np.testing.assert_allclose(w[sel], int(num) / int(den), rtol=1e-15, atol=0)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("RT", [1.0 / 3.0, 0.2, 0.45])
def test_weight_isotropy(D, RT):
    """Sum w = 1, sum w c_a c_b = RT delta_ab (any RT); at RT = 1/3 the fourth moment is
    isotropic, RT^2 (d_ab d_cd + d_ac d_bd + d_ad d_bc)."""
    c, _ = oracle.lattice(D)
    c = c[:, :D].astype(float)
    w = oracle.weights(D, RT)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), RT * np.eye(D), atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-17)
    if abs(RT - 1.0 / 3.0) < 1e-15:
        m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
        I = np.eye(D)
        iso = RT * RT * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                         + np.einsum("ad,bc->abcd", I, I))
        np.testing.assert_allclose(m4, iso, atol=1e-16)


def _moments(c, f):
    return (f.sum(), np.einsum("ia,i->a", c, f), np.einsum("ia,ib,i->ab", c, c, f),
            np.einsum("ia,ib,ic,i->abc", c, c, c, f))


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("RT", [1.0 / 3.0, 0.25])
def test_equilibrium_moments(D, RT):
    """Eqs. (Pi_0_eq)-(Pi_2_eq) and the third moment with its diagonal anomaly
    (Pi_3_prod_generic) for xi = v/eps, P = xi^2 + RT."""
    rng = np.random.default_rng(1)
    c, _ = oracle.lattice(D)
    c = c[:, :D].astype(float)
    for _ in range(20):
        eps = rng.uniform(0.2, 1.0)
        rho = rng.uniform(0.8, 1.2)
        v = rng.uniform(-0.1, 0.1, D)
        xi = v / eps
        P = xi * xi + RT
        f = oracle.product_form(D, eps, rho, xi, P)
        m0, m1, m2, m3 = _moments(c, f)
        I = np.eye(D)
        assert abs(m0 - eps * rho) < 1e-15
        np.testing.assert_allclose(m1, rho * v, atol=2e-16)
        np.testing.assert_allclose(m2, rho * np.outer(v, v) / eps + eps * rho * RT * I,
                                   atol=2e-16)
        t3 = (np.einsum("a,b,c->abc", xi, xi, xi)
              + RT * (np.einsum("a,bc->abc", xi, I) + np.einsum("b,ac->abc", xi, I)
                      + np.einsum("c,ab->abc", xi, I)))
        diag = np.zeros((D, D, D))
        for a in range(D):
            diag[a, a, a] = (1.0 - 3.0 * RT - xi[a] ** 2) * xi[a]
        np.testing.assert_allclose(m3, eps * rho * (t3 + diag), atol=5e-16)


@pytest.mark.parametrize("D", [2, 3])
def test_shifted_equilibrium_moments(D):
    """Eq. (Pi_2_prod_general) for arbitrary (xi*, P*): sum c_a^2 f = eps rho P*_aa and
    sum c_a c_b f = eps rho xi*_a xi*_b off the diagonal; sum c f = eps rho xi*."""
    rng = np.random.default_rng(2)
    c, _ = oracle.lattice(D)
    c = c[:, :D].astype(float)
    for _ in range(20):
        eps, rho = rng.uniform(0.2, 1.0), rng.uniform(0.8, 1.2)
        xs = rng.uniform(-0.2, 0.2, D)
        Ps = xs * xs + 1.0 / 3.0 + rng.uniform(-0.05, 0.05, D)
        f = oracle.product_form(D, eps, rho, xs, Ps)
        m0, m1, m2, _ = _moments(c, f)
        assert abs(m0 - eps * rho) < 1e-15
        np.testing.assert_allclose(m1, eps * rho * xs, atol=2e-16)
        expect = eps * rho * np.outer(xs, xs)
        np.fill_diagonal(expect, eps * rho * Ps)
        np.testing.assert_allclose(m2, expect, atol=2e-16)


def test_drag_solve_satisfies_quadratic():
    """Appendix D, eq. (v_quadratic): c1 v + c2 |v| v = v' with c1 = 1 + mu_D/2, c2 = mu_F/2;
    the root is the non-negative one and v is parallel to v'."""
    rng = np.random.default_rng(3)
    for D in (2, 3):
        for _ in range(200):
            v0 = rng.normal(0, 10 ** rng.uniform(-8, -1), D)
            muD = 10 ** rng.uniform(-6, 2) * rng.integers(0, 2)
            muF = 10 ** rng.uniform(-4, 2) * rng.integers(0, 2)
            v = oracle.drag_solve(v0, muD, muF)
            c1, c2 = 1 + 0.5 * muD, 0.5 * muF
            res = c1 * v + c2 * np.linalg.norm(v) * v - v0
            assert np.linalg.norm(res) <= 1e-14 * np.linalg.norm(v0)
            assert np.dot(v, v0) >= 0
    assert np.all(oracle.drag_solve(np.zeros(3), 2.0, 3.0) == 0)
    v0 = np.array([0.3, -0.1])
    np.testing.assert_allclose(oracle.drag_solve(v0, 4.0, 0.0), v0 / 3.0, rtol=1e-15)


def _oracle_box(D, n, eps, kappa=None, cf=None, mask=None, **kw):
    shape = (1, n, n) if D == 2 else (n, n, n)
    e = np.broadcast_to(eps, shape).astype(float).copy()
    k = np.full(shape, np.inf) if kappa is None else np.broadcast_to(kappa, shape).copy()
    f = np.zeros(shape) if cf is None else np.broadcast_to(cf, shape).copy()
    return oracle.Oracle(oracle.OracleConfig(D=D, eps=e, kappa=k, cf=f, mask=mask, **kw))


def _spectral_grad(f, axis, L):
    k = np.fft.fftfreq(f.shape[axis], d=1.0) * 2 * np.pi
    sh = [1] * f.ndim
    sh[axis] = -1
    return np.real(np.fft.ifft(1j * k.reshape(sh) * np.fft.fft(f, axis=axis), axis=axis))


@pytest.mark.parametrize("pow_", [0, -1, 1])
def test_delta_nu_expansion_matches_divergence_form(pow_):
    """Eq. (porosity_correction_expanded) must equal the divergence form (porosity_correction)
    Delta_nu(m) = div[nu_eff(eps)(m (x) grad eps + grad eps (x) m)] up to the O(h^2) error of the
    central differences.  The reference is an independent spectral evaluation of the divergence
    form on smooth periodic fields; the error must fall ~4x per grid doubling."""
    errs = []
    for n in (32, 64, 128):
        x = (np.arange(n) + 0.0) * (2 * np.pi / n)
        X, Y = np.meshgrid(x, x, indexing="xy")  # [y, x]
        eps = 0.6 + 0.25 * np.sin(X + 0.3) * np.cos(2 * Y)
        m = np.stack([0.3 * np.cos(X) * np.sin(Y + 0.5), 0.2 * np.sin(2 * X + Y)])
        # the oracle works in lattice units (dx = 1); the fields above have period n cells
        nu_ref = 0.1
        o = _oracle_box(2, n, eps[None], nu_eff_ref=nu_ref, nu_eff_pow=pow_)
        got = o.delta_nu(m[:, None])[:, 0]
        nu = nu_ref * eps ** pow_
        ge = [_spectral_grad(eps, 1, n), _spectral_grad(eps, 0, n)]
        flux = [[nu * (m[a] * ge[b] + ge[a] * m[b]) for b in range(2)] for a in range(2)]
        ref = np.stack([_spectral_grad(flux[a][0], 1, n) + _spectral_grad(flux[a][1], 0, n)
                        for a in range(2)])
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.6 and errs[1] / errs[2] > 3.8, errs


def test_porosity_derivatives_are_second_order():
    """The central differences of eps (Sec. 3.5, last paragraph) converge at second order to the
    analytic gradient and Hessian of a smooth periodic field, in 3D including mixed terms."""
    errs = []
    for n in (16, 32, 64):
        h = 2 * np.pi / n
        z, y, x = np.meshgrid(*(np.arange(n) * h,) * 3, indexing="ij")
        eps = 0.6 + 0.2 * np.sin(x) * np.cos(y) * np.sin(z + 0.4)
        o = _oracle_box(3, n, eps)
        ge, H = o.porosity_derivatives()
        ex = 0.2 * np.cos(x) * np.cos(y) * np.sin(z + 0.4) * h
        exy = -0.2 * np.cos(x) * np.sin(y) * np.sin(z + 0.4) * h * h
        exx = -0.2 * np.sin(x) * np.cos(y) * np.sin(z + 0.4) * h * h
        assert np.array_equal(H[0, 1], H[1, 0])
        errs.append(max(np.abs(ge[0] - ex).max() / h, np.abs(H[0, 1] - exy).max() / h ** 2,
                        np.abs(H[0, 0] - exx).max() / h ** 2))
    assert errs[0] / errs[1] > 3.8 and errs[1] / errs[2] > 3.9, errs


@pytest.mark.parametrize("H", [6, 2])
def test_one_sided_differences_next_to_walls(H):
    """Sec. 3.5, last paragraph: next to a boundary the moment-field derivatives are second-order
    one-sided differences (exact on quadratics); with a single fluid neighbour the first-order
    fallback is exact on linear fields.  Checked through Delta_nu with eps linear in y and
    m = (m_x(y), 0): Delta_nu(m)_x = nu m_x'(y) eps'(y) exactly, on every fluid row."""
    ny = H + 2
    y = np.arange(ny, dtype=float)
    eps = (0.5 + 0.01 * y)[None, :, None] * np.ones((1, ny, 3))
    mask = np.zeros((1, ny, 3), dtype=np.uint8)
    mask[:, 0] = mask[:, -1] = 1
    o = oracle.Oracle(oracle.OracleConfig(D=2, eps=eps, kappa=np.full(eps.shape, np.inf),
                                          cf=np.zeros(eps.shape), mask=mask, nu_eff_ref=0.2))
    cq = 0.0 if H == 2 else 3e-3
    mx = 0.1 + 0.02 * y + cq * y * y
    m = np.zeros((2, 1, ny, 3))
    m[0] = mx[None, :, None]
    got = o.delta_nu(m)
    expect = 0.2 * (0.02 + 2 * cq * y) * 0.01
    np.testing.assert_allclose(got[0, 0, 1:-1, 1], expect[1:-1], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(got[1, 0, 1:-1, 1], 0.0, atol=1e-18)
