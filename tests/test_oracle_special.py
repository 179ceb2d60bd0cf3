"""Pins for the oracle's special functions: spherical Bessel j_l, spherical harmonics Y_lm
and Gaunt coefficients, against closed forms, library routines (scipy, sympy), identities
the paper states (the addition theorem in section 3.1) and brute-force quadrature."""
import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y, spherical_jn

pytestmark = pytest.mark.usefixtures("oracle_lib")

XS = [1e-8, 1e-5, 1e-3, 0.05, 0.3, 0.5, 1.0, 1.7, 2.5, np.pi, 4.0, 5.3, 2 * np.pi, 6.7, 9.0, 15.0, 27.5, 50.0]


def _close(x, ref, rel=1e-13, abs_=2e-16):
    return np.all(np.abs(x - ref) <= rel * np.abs(ref) + abs_)


@pytest.mark.parametrize("x", XS)
def test_bessel_vs_scipy(oracle_lib, x):
    j, dj = oracle_lib.sph_bessel(14, x)
    ls = np.arange(15)
    assert _close(j, spherical_jn(ls, x))
    assert _close(dj, spherical_jn(ls, x, derivative=True), rel=1e-12)


@pytest.mark.parametrize("x", [1.0, 1.3, 3.0, 7.7, 20.0])  # the closed forms cancel badly below 1
def test_bessel_closed_forms(oracle_lib, x):
    j, dj = oracle_lib.sph_bessel(2, x)
    s, c = np.sin(x), np.cos(x)
    j0 = s / x
    j1 = s / x ** 2 - c / x
    j2 = (3 / x ** 2 - 1) * s / x - 3 * c / x ** 2
    assert _close(j, np.array([j0, j1, j2]), rel=1e-13, abs_=1e-15)
    # j0' = cos/x - sin/x^2 ; j1' = j0 - 2 j1 / x
    assert abs(dj[0] - (c / x - s / x ** 2)) < 1e-14
    assert abs(dj[1] - (j0 - 2 * j1 / x)) < 1e-14


def test_bessel_tabulated(oracle_lib):
    j, dj = oracle_lib.sph_bessel(10, 0.5)
    assert abs(j[0] - 0.958851077208406) < 1e-15
    assert abs(j[1] - 0.1625370306360667) < 1e-15
    j, dj = oracle_lib.sph_bessel(10, 3.0)
    assert abs(j[2] - 0.29863749707573356) < 1e-15
    j, dj = oracle_lib.sph_bessel(10, 1.0)
    assert abs(j[10] / 7.116552640047341e-11 - 1) < 1e-13     # small x, large l


@pytest.mark.parametrize("x", [1e-9, 1e-4, 1e-2])
def test_bessel_small_x_series(oracle_lib, x):
    j, dj = oracle_lib.sph_bessel(10, x)
    for l in range(11):
        dfact = np.prod(np.arange(1, 2 * l + 2, 2, dtype=float))
        lead = x ** l / dfact * (1 - x * x / (2 * (2 * l + 3)) + x ** 4 / (8 * (2 * l + 3) * (2 * l + 5)))
        assert abs(j[l] - lead) <= 1e-12 * abs(lead) + 1e-300


def test_bessel_zero(oracle_lib):
    j, dj = oracle_lib.sph_bessel(6, 0.0)
    assert j[0] == 1.0 and np.all(j[1:] == 0.0)
    assert abs(dj[1] - 1 / 3) < 1e-16 and dj[0] == 0.0


def test_bessel_derivative_recurrence(oracle_lib):
    # j_l' = (l j_{l-1} - (l+1) j_{l+1}) / (2l+1), a different identity than the oracle uses
    for x in [0.3, 2.0, 6.0, 11.0]:
        j, dj = oracle_lib.sph_bessel(12, x)
        for l in range(1, 12):
            alt = (l * j[l - 1] - (l + 1) * j[l + 1]) / (2 * l + 1)
            assert abs(dj[l] - alt) <= 1e-13 * max(abs(alt), 1e-3 * abs(j[l - 1])) + 1e-17


def _angles(v):
    r = np.linalg.norm(v)
    return np.arccos(np.clip(v[2] / r, -1, 1)), np.arctan2(v[1], v[0])


def test_ylm_vs_scipy(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(60):
        v = rng.standard_normal(3) * rng.uniform(0.1, 10)
        y = oracle_lib.ylm(10, v)
        th, ph = _angles(v)
        for l in range(11):
            for m in range(-l, l + 1):
                assert abs(y[l * l + l + m] - sph_harm_y(l, m, th, ph)) < 5e-15


def test_ylm_closed_forms(oracle_lib):
    rng = np.random.default_rng(6)
    for _ in range(20):
        v = rng.standard_normal(3)
        x, y_, z = v / np.linalg.norm(v)
        y = oracle_lib.ylm(2, v)
        assert abs(y[0] - 0.5 / np.sqrt(np.pi)) < 1e-16
        assert abs(y[2] - np.sqrt(3 / (4 * np.pi)) * z) < 1e-15
        assert abs(y[3] - (-np.sqrt(3 / (8 * np.pi)) * (x + 1j * y_))) < 1e-15
        assert abs(y[1] - (np.sqrt(3 / (8 * np.pi)) * (x - 1j * y_))) < 1e-15
        assert abs(y[6] - np.sqrt(5 / (16 * np.pi)) * (3 * z * z - 1)) < 1e-15
        assert abs(y[7] - (-np.sqrt(15 / (8 * np.pi)) * z * (x + 1j * y_))) < 1e-15
        assert abs(y[8] - np.sqrt(15 / (32 * np.pi)) * (x + 1j * y_) ** 2) < 1e-15


def test_ylm_poles_and_zero_vector(oracle_lib):
    for v, sgn in (([0, 0, 2.0], 1), ([0, 0, -3.0], -1), ([0, 0, 0.0], 1)):
        y = oracle_lib.ylm(8, v)
        for l in range(9):
            for m in range(-l, l + 1):
                ref = np.sqrt((2 * l + 1) / (4 * np.pi)) * (sgn ** l) if m == 0 else 0.0
                assert abs(y[l * l + l + m] - ref) < 1e-14


def test_ylm_addition_theorem(oracle_lib):
    """sum_m Y_lm(u) conj(Y_lm(v)) = (2l+1)/(4 pi) P_l(u.v): the identity the paper uses
    for FLEUR's reduction of S (section 3.1)."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        u, v = rng.standard_normal(3), rng.standard_normal(3)
        yu, yv = oracle_lib.ylm(10, u), oracle_lib.ylm(10, v)
        c = np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v)
        for l in range(11):
            sl = slice(l * l, (l + 1) ** 2)
            s = np.sum(yu[sl] * np.conj(yv[sl]))
            assert abs(s - (2 * l + 1) / (4 * np.pi) * eval_legendre(l, c)) < 1e-14 * (2 * l + 1)
            assert abs(np.sum(np.abs(yu[sl]) ** 2) - (2 * l + 1) / (4 * np.pi)) < 1e-14 * (2 * l + 1)


def _sphere_quadrature(n_theta, n_phi):
    z, w = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    Z, P = np.meshgrid(z, ph, indexing="ij")
    W = np.outer(w, np.full(n_phi, 2 * np.pi / n_phi))
    st = np.sqrt(1 - Z * Z)
    pts = np.stack([st * np.cos(P), st * np.sin(P), Z], -1).reshape(-1, 3)
    return pts, W.reshape(-1)


def test_ylm_orthonormal_by_quadrature(oracle_lib):
    pts, w = _sphere_quadrature(12, 24)                 # exact for the degree-16 products below
    Y = np.stack([oracle_lib.ylm(7, p) for p in pts])   # (npts, 64)
    gram = (Y.conj().T * w) @ Y
    assert np.abs(gram - np.eye(64)).max() < 1e-13


def test_gaunt_vs_sympy(oracle_lib):
    from sympy.physics.wigner import gaunt
    rng = np.random.default_rng(8)
    checked = 0
    for _ in range(400):
        l, lp, lpp = int(rng.integers(0, 11)), int(rng.integers(0, 11)), int(rng.integers(0, 9))
        m, mpp = int(rng.integers(-l, l + 1)), int(rng.integers(-lpp, lpp + 1))
        mp = m + mpp
        if abs(mp) > lp:
            continue
        ref = float((-1) ** mp * gaunt(lp, l, lpp, -mp, m, mpp))
        assert abs(oracle_lib.gaunt(l, m, lp, mp, lpp, mpp) - ref) < 2e-15
        checked += 1
    assert checked > 150


@pytest.mark.parametrize("idx,val", [
    ((1, 0, 1, 0, 2, 0), 1 / np.sqrt(5 * np.pi)),
    ((1, 1, 1, 1, 2, 0), -1 / (2 * np.sqrt(5 * np.pi))),
    ((2, 1, 1, 0, 1, -1), None),
    ((1, 0, 1, 1, 1, 1), 0.0),
])
def test_gaunt_tabulated(oracle_lib, idx, val):
    from sympy.physics.wigner import gaunt
    l, m, lp, mp, lpp, mpp = idx
    g = oracle_lib.gaunt(l, m, lp, mp, lpp, mpp)
    if val is None:
        val = float((-1) ** mp * gaunt(lp, l, lpp, -mp, m, mpp))
    assert abs(g - val) < 1e-15


def test_gaunt_selection_rules_and_l0(oracle_lib):
    for l in range(6):
        for m in range(-l, l + 1):
            for lp in range(6):
                for mp in range(-lp, lp + 1):
                    g0 = oracle_lib.gaunt(l, m, lp, mp, 0, 0)
                    assert abs(g0 - ((l == lp and m == mp) / np.sqrt(4 * np.pi))) < 1e-15
                    for lpp in range(5):
                        for mpp in range(-lpp, lpp + 1):
                            g = oracle_lib.gaunt(l, m, lp, mp, lpp, mpp)
                            allowed = (mp == m + mpp) and ((l + lp + lpp) % 2 == 0) and abs(l - lpp) <= lp <= l + lpp
                            if not allowed:
                                assert g == 0.0


def test_gaunt_by_quadrature(oracle_lib):
    """G_{L,L',L''} = int conj(Y_L') Y_L Y_L'' by brute-force product quadrature with scipy's Y."""
    pts, w = _sphere_quadrature(14, 28)
    th = np.arccos(np.clip(pts[:, 2], -1, 1))
    ph = np.arctan2(pts[:, 1], pts[:, 0])
    rng = np.random.default_rng(9)
    for _ in range(120):
        l, lp, lpp = int(rng.integers(0, 8)), int(rng.integers(0, 8)), int(rng.integers(0, 7))
        m, mp, mpp = int(rng.integers(-l, l + 1)), int(rng.integers(-lp, lp + 1)), int(rng.integers(-lpp, lpp + 1))
        f = np.conj(sph_harm_y(lp, mp, th, ph)) * sph_harm_y(l, m, th, ph) * sph_harm_y(lpp, mpp, th, ph)
        q = np.sum(w * f)
        assert abs(q - oracle_lib.gaunt(l, m, lp, mp, lpp, mpp)) < 1e-14
