"""Pins of the oracle's radial functions and radial integrals (section 2.2, eq. simp_Schr;
appendix A.2, eqs. nonsph_integrals and the Wronskian of the coefficients), in Hartree units.

Each pin checks the oracle against something other than itself:
  * the regular Coulomb solution r^(l+1) e^(-kappa r) M(l+1-Z/kappa, 2l+2, 2 kappa r) (scipy's
    confluent hypergeometric function) and the free solution r j_l(k r) (scipy's spherical Bessel);
  * the energy derivative against a central finite difference in E of the normalised solution;
  * the Wronskian identity udot u' - u udot' = 2 / R^2 that follows from normalisation;
  * fourth-order convergence of the outward integration;
  * the Simpson integral against scipy's adaptive quadrature of closed-form integrands;
  * invariants of the integral tables (symmetry, normalisation, orthogonality).
"""
import numpy as np
import pytest
from scipy.integrate import quad, simpson
from scipy.special import hyp1f1, spherical_jn

import oracle


def coulomb_p(r, l, z, e):
    kappa = np.sqrt(-2.0 * e)
    return r ** (l + 1) * np.exp(-kappa * r) * hyp1f1(l + 1 - z / kappa, 2 * l + 2, 2 * kappa * r)


def _normalised(f, r0, rmax):
    return np.sqrt(quad(lambda x: f(x) ** 2, r0, rmax, epsabs=1e-15, epsrel=1e-13, limit=200)[0])


R0, RMT, Z, E = 1e-6, 2.2, 3.0, -0.7


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_coulomb_regular_solution(l):
    n_r = 3201
    r = oracle.radial_mesh(n_r, R0, RMT)
    P, Pd, b = oracle.radial(n_r, R0, RMT, -Z / r, l, E)
    re = r[::2]
    nn = _normalised(lambda x: coulomb_p(x, l, Z, E), R0, RMT)
    ex = coulomb_p(re, l, Z, E) / nn
    assert np.max(np.abs(P - ex)) / np.max(np.abs(ex)) < 1e-7
    # boundary values: u = P / R and u' from the closed form's derivative
    h = 1e-5
    uex = coulomb_p(RMT, l, Z, E) / nn / RMT
    dpex = (coulomb_p(RMT + h, l, Z, E) - coulomb_p(RMT - h, l, Z, E)) / (2 * h) / nn
    duex = dpex / RMT - coulomb_p(RMT, l, Z, E) / nn / RMT ** 2
    assert b["u"] == pytest.approx(uex, rel=1e-6)
    assert b["du"] == pytest.approx(duex, rel=1e-5)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 6])
def test_free_solution(l):
    n_r, r0, rmax, k = 3201, 1e-6, 2.5, 1.7
    r = oracle.radial_mesh(n_r, r0, rmax)
    P, _, b = oracle.radial(n_r, r0, rmax, np.zeros(n_r), l, 0.5 * k * k)
    re = r[::2]
    f = lambda x: x * spherical_jn(l, k * x)
    ex = f(re) / _normalised(f, r0, rmax)
    assert np.max(np.abs(P - ex)) / np.max(np.abs(ex)) < 1e-6


def test_hydrogen_bound_state_log_derivative():
    """At the 1s eigenvalue E = -Z^2/2 the solution is r e^(-Z r): u'/u = -Z at any radius.
    (Outward integration of a decaying solution amplifies the step error by about e^(2 Z R),
    hence the small radius.)"""
    n_r, rmax = 2001, 1.2
    r = oracle.radial_mesh(n_r, R0, rmax)
    _, _, b = oracle.radial(n_r, R0, rmax, -Z / r, 0, -0.5 * Z * Z)
    assert b["du"] / b["u"] == pytest.approx(-Z, rel=1e-6)


def test_fourth_order_convergence():
    l = 1
    errs = []
    for n_r in (401, 801, 1601):
        r = oracle.radial_mesh(n_r, R0, RMT)
        P, _, _ = oracle.radial(n_r, R0, RMT, -Z / r, l, E)
        ex = coulomb_p(r[::2], l, Z, E) / _normalised(lambda x: coulomb_p(x, l, Z, E), R0, RMT)
        errs.append(np.max(np.abs(P - ex)))
    for a, c in zip(errs, errs[1:]):
        assert 12.0 < a / c < 20.0


@pytest.mark.parametrize("l", [0, 1, 4])
def test_energy_derivative_is_finite_difference(l):
    """Pd and the boundary values of udot equal d/dE of the normalised P and of u(R), u'(R)."""
    n_r, d = 1601, 1e-4
    r = oracle.radial_mesh(n_r, R0, RMT)
    v = -Z / r + 0.3 * (r / RMT) ** 2
    P, Pd, b = oracle.radial(n_r, R0, RMT, v, l, E)
    Pp, _, bp = oracle.radial(n_r, R0, RMT, v, l, E + d)
    Pm, _, bm = oracle.radial(n_r, R0, RMT, v, l, E - d)
    assert np.max(np.abs(Pd - (Pp - Pm) / (2 * d))) / np.max(np.abs(Pd)) < 1e-7
    assert b["ud"] == pytest.approx((bp["u"] - bm["u"]) / (2 * d), rel=1e-7, abs=1e-8)
    assert b["dud"] == pytest.approx((bp["du"] - bm["du"]) / (2 * d), rel=1e-7, abs=1e-8)
    # ||udot||^2 is the integral of Pd^2 dr: scipy's Simpson rule in x = ln r (dr = r dx)
    re = r[::2]
    assert b["ud_norm2"] == pytest.approx(simpson(Pd * Pd * re, x=np.log(re)), rel=1e-12)


@pytest.mark.parametrize("l", [0, 2, 5])
def test_wronskian_identity(l):
    """-1/2 (P Pd' - Pd P') integrated from the origin equals the norm of P (= 1), so
    udot u' - u udot' = 2 / R^2 for the normalised functions (Hartree units)."""
    n_r = 3201
    r = oracle.radial_mesh(n_r, R0, RMT)
    v = -Z / r + Z * (3 * RMT ** 2 - r ** 2) / (2 * RMT ** 3)
    _, _, b = oracle.radial(n_r, R0, RMT, v, l, -0.2 + 0.1 * l)
    w = b["ud"] * b["du"] - b["u"] * b["dud"]
    assert w == pytest.approx(2.0 / RMT ** 2, rel=1e-5)


@pytest.mark.parametrize("n", [0, 1, 3])
def test_simpson_integral_against_quadrature(n):
    """The integral of P v P dr on the log mesh (weights r dx) against adaptive quadrature."""
    n_r = 3201
    r = oracle.radial_mesh(n_r, R0, RMT)[::2]
    fa = coulomb_p(r, 1, Z, E)
    fb = coulomb_p(r, 2, Z, E)
    v = (r / RMT) ** n * np.cos(r)
    got = oracle.radial_integral(n_r, R0, RMT, fa, v, fb)
    ref = quad(lambda x: coulomb_p(x, 1, Z, E) * (x / RMT) ** n * np.cos(x) * coulomb_p(x, 2, Z, E),
               R0, RMT, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    assert got == pytest.approx(ref, rel=5e-6)


def test_setup_tables_invariants():
    """Symmetry of I^{uu}, I^{udot udot}; I^{udot u} is I^{u udot} transposed; with v_00 = c on
    the L''=0 slot: I^{uu}_{ll} = c, I^{u udot}_{ll} = 0 and I^{udot udot}_{ll} = c ||udot||^2."""
    n_r, lpot = 801, 2
    rmt = np.array([2.0, 2.4])
    r0 = np.array([1e-5, 2e-6])
    lmax = np.array([3, 2])
    nlp = (lpot + 1) ** 2
    v0, vlm, e_l = [], [], np.array([[-0.4, -0.3, -0.2, 0.1], [-0.5, -0.1, 0.2, 0.0]])
    c = 0.37
    for t in range(2):
        r = oracle.radial_mesh(n_r, r0[t], rmt[t])
        v0.append(-(4.0 + 2 * t) / r)
        comp = np.zeros((nlp, n_r))
        comp[0] = c
        for L in range(1, nlp):
            comp[L] = 0.1 * L * (r / rmt[t]) ** 2 * np.exp(-r)
        comp[1] = -comp[3]                     # reality rule for (1, -1) from (1, 1)
        comp[4] = comp[8]                      # (2, -2) from (2, 2)
        comp[5] = -comp[7]                     # (2, -1) from (2, 1)
        vlm.append(comp)
    out = oracle.radial_setup(n_r, r0, rmt, v0, e_l, lmax, vlm, lpot)
    for t in range(2):
        n = lmax[t] + 1
        uu = out["i_uu"][t, :n, :n]
        dd = out["i_dd"][t, :n, :n]
        assert np.allclose(uu, uu.transpose(1, 0, 2), rtol=0, atol=1e-15)
        assert np.allclose(dd, dd.transpose(1, 0, 2), rtol=0, atol=1e-15)
        assert np.allclose(out["i_du"][t, :n, :n], out["i_ud"][t, :n, :n].transpose(1, 0, 2), rtol=0, atol=1e-15)
        for l in range(n):
            assert out["i_uu"][t, l, l, 0] == pytest.approx(c, rel=1e-13)
            assert abs(out["i_ud"][t, l, l, 0]) < 1e-13
            assert out["i_dd"][t, l, l, 0] == pytest.approx(c * out["ud_norm2"][t, l], rel=1e-13)
            w = out["ud"][t, l] * out["du"][t, l] - out["u"][t, l] * out["dud"][t, l]
            assert w == pytest.approx(2.0 / rmt[t] ** 2, rel=1e-4)
