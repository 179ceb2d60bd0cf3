"""Pins of the oracle's interstitial terms and of its generalized eigensolve (section 2.3: eq.
basis_function, whose interstitial branch is the plane wave exp(i K_t.r)/sqrt(Omega); eq. HS_Mat
over the cell minus the muffin-tin spheres; eq. matrix_kohnsham).

Each check is independent of the closed form the oracle evaluates:
  * the ball integral of a plane wave by a product Gauss quadrature in spherical coordinates
    around the atom (no Bessel function), which also fixes the sign of the phase exp(i G.x_a);
  * the cell-minus-spheres integral by a midpoint grid over the whole cell, with the spheres'
    periodic images (an atom near a corner), which fixes the meaning of the region;
  * the diagonal = the interstitial volume fraction;
  * Hermiticity, and positive semidefiniteness of S^I (a Gram matrix of plane waves on a region);
  * spheres of vanishing radius: H^I c = eps S^I c has the free-electron levels |K_t|^2 / 2 + v;
  * the eigenpairs solve H c = eps S c with c^H S c = 1, and agree with a Cholesky reduction done
    with numpy."""
import numpy as np
import pytest

import oracle
import synthcells


def _one_atom(pos, R=1.7, a=7.0, n_g=40, seed=3):
    return synthcells.custom_cell("int1", a, np.asarray([pos], float), np.zeros(1, np.int32), [3], [R], 2, n_g,
                                  [seed])


def _ball_quadrature(G, x, R, n=48, nphi=96):
    """(integral over |r - x| < R of exp(i G.r) dr) by Gauss-Legendre in the radius and in cos(theta)
    and the trapezoid rule in phi (exact for the entire integrand to rounding at these orders)."""
    zr, wr = np.polynomial.legendre.leggauss(n)
    rho, wrho = 0.5 * R * (zr + 1.0), 0.5 * R * wr
    mu, wmu = np.polynomial.legendre.leggauss(n)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - mu ** 2)
    dirs = np.stack([st[:, None] * np.cos(phi)[None, :], st[:, None] * np.sin(phi)[None, :],
                     np.broadcast_to(mu[:, None], (n, nphi))], axis=-1)          # (n_mu, n_phi, 3)
    gd = dirs @ G                                                                  # (n_mu, n_phi)
    ph = np.exp(1j * rho[:, None, None] * gd[None])                                # (n_r, n_mu, n_phi)
    w = (wrho * rho ** 2)[:, None, None] * wmu[None, :, None] * (2.0 * np.pi / nphi)
    return np.exp(1j * G @ x) * np.sum(w * ph)


def test_ball_integral_by_quadrature():
    x = np.array([1.3, 5.9, 2.2])
    cell = _one_atom(x)
    rng = np.random.default_rng(5)
    rows = rng.choice(cell.n_g(0), 12, replace=False)
    cols = rng.choice(cell.n_g(0), 12, replace=False)
    _, S = oracle.interstitial_block(cell, 0, rows, cols)
    g = cell.gvecs[0]
    for a, r in enumerate(rows):
        for b, c in enumerate(cols):
            G = g[c] - g[r]
            want = (1.0 if r == c else 0.0) - _ball_quadrature(G, x, cell.rmt[0]) / cell.omega
            assert abs(S[a, b] - want) < 1e-14, (r, c)


def test_diagonal_is_the_interstitial_volume_fraction():
    cell = synthcells.config(3, n_k=1)
    _, S = oracle.interstitial_block(cell, 0, np.arange(20), np.arange(20))
    frac = 1.0 - np.sum(4.0 * np.pi / 3.0 * cell.rmt[cell.atom_type] ** 3) / cell.omega
    assert np.allclose(np.diag(S), frac, rtol=0, atol=1e-14)


def test_cell_minus_spheres_on_a_grid():
    """Midpoint rule over the cell with the spheres (and their periodic images) cut out: one atom
    near a corner, so that its sphere crosses three cell faces.  The grid rule on a discontinuous
    integrand converges slowly; 160^3 points give about 3e-5 against entries of 1e-2."""
    a = 6.0
    pos = np.array([[0.4, 0.3, 5.7], [3.1, 2.9, 3.3]])
    cell = synthcells.custom_cell("grid", a, pos, np.array([0, 1], np.int32), [2, 2], [1.3, 1.0], 2, 30, [9])
    n = 160
    h = a / n
    ax = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    inside = np.zeros(X.shape, bool)
    for p, R in zip(pos, cell.rmt[cell.atom_type]):
        d = [np.abs(C - pc) for C, pc in ((X, p[0]), (Y, p[1]), (Z, p[2]))]
        d = [np.minimum(di, a - di) for di in d]                        # minimum image in a cubic cell
        inside |= d[0] ** 2 + d[1] ** 2 + d[2] ** 2 < R * R
    keep = ~inside
    g = cell.gvecs[0]
    rows, cols = np.array([0, 3, 7, 11]), np.array([1, 3, 8, 20])
    _, S = oracle.interstitial_block(cell, 0, rows, cols)
    for i, r in enumerate(rows):
        for j, c in enumerate(cols):
            G = g[c] - g[r]
            ph = np.exp(1j * (G[0] * X[keep] + G[1] * Y[keep] + G[2] * Z[keep]))
            want = ph.sum() * h ** 3 / cell.omega
            assert abs(S[i, j] - want) < 2e-4, (r, c, S[i, j], want)


def test_hermitian_and_positive_semidefinite():
    cell = synthcells.config(1)
    assert synthcells.min_sphere_gap(cell) > 0
    idx = np.random.default_rng(2).choice(cell.n_g(0), 200, replace=False)
    H, S = oracle.interstitial_block(cell, 0, idx, idx, v_int=0.3)
    assert np.abs(S - S.conj().T).max() < 1e-15
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    lam = np.linalg.eigvalsh(S)
    assert lam.min() > -1e-13 * lam.max()
    # H^I = (K'.K / 2 + v) S^I: the diagonal is the interstitial kinetic energy of the plane wave
    K = cell.kpts[0] + cell.gvecs[0][idx]
    frac = S[0, 0].real
    assert np.allclose(np.diag(H).real, (0.5 * np.sum(K * K, axis=1) + 0.3) * frac, rtol=1e-14, atol=0)


def test_free_electron_limit():
    """Spheres of radius 1e-4: S^I = 1 - O(R^3), and H^I c = eps S^I c gives |K_t|^2 / 2 + v."""
    cell = synthcells.custom_cell("free", 7.5, np.array([[1.0, 2.0, 3.0], [4.0, 5.5, 6.0]]),
                                  np.zeros(2, np.int32), [2], [1e-4], 2, 60, [4])
    H, S = oracle.interstitial_block(cell, 0, v_int=-0.2)
    w, _ = oracle.eigh_generalized(H, S)
    K = cell.kpts[0] + cell.gvecs[0]
    want = np.sort(0.5 * np.sum(K * K, axis=1) - 0.2)
    assert np.allclose(w, want, rtol=0, atol=1e-10)


@pytest.fixture(scope="module")
def total_c0():
    cell = synthcells.config_separated(0)
    H, S = oracle.hs_total(cell, 0, v_int=0.1)
    return cell, H, S


def test_total_overlap_is_positive_definite(total_c0):
    """Muffin-tin S (rank <= 2K, singular here: N = 300 > 196) plus the interstitial S."""
    cell, H, S = total_c0
    assert cell.n_g(0) > 2 * cell.k_rows()
    lam = np.linalg.eigvalsh(S)
    assert lam.min() > 1e-6 * lam.max()
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(H).max()


def test_generalized_eigenpairs(total_c0):
    _, H, S = total_c0
    w, C = oracle.eigh_generalized(H, S)
    assert np.all(np.diff(w) >= 0)
    R = H @ C - (S @ C) * w[None, :]
    assert np.abs(R).max() < 1e-11 * np.abs(H).max() * np.abs(C).max()
    assert np.abs(C.conj().T @ S @ C - np.eye(len(w))).max() < 1e-11
    # the same eigenvalues from a Cholesky reduction done here with numpy
    Lc = np.linalg.cholesky(S)
    Li = np.linalg.inv(Lc)
    w2 = np.linalg.eigvalsh(Li @ H @ Li.conj().T)
    assert np.abs(w - w2).max() < 1e-10 * np.abs(w).max()
