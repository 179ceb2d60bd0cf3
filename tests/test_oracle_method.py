"""Pins for the oracle's matching coefficients, T matrices, S and H.

Each check is anchored outside the oracle's own code: scipy's j_l and Y_lm, the C^1
matching conditions the coefficients are defined by (appendix A.1), the plane-wave
continuity they imply, FLEUR's Legendre form of S (section 3.1, with its prefactor
corrected), invariants (Hermiticity, positive semidefiniteness, rotation invariance of S),
closed forms for special potentials, and a brute-force angular quadrature of the
non-spherical matrix elements written from eq. h_expanded_basis."""
import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y, spherical_jn

import synthcells

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _tiny(seed=11, lmax=(3, 2), lpot=2, n_g=14, rotations="random", a=7.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, a, size=(2, 3))
    return synthcells.custom_cell("tiny", a, pos, np.array([0, 1], np.int32), list(lmax), [1.6, 1.9], lpot, n_g,
                                  [seed], rotations=rotations)


def _mixed(seed=12, n_g=90):
    """3 atoms, 2 types with different l_max, random rotations."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 9.0, size=(3, 3))
    return synthcells.custom_cell("mixed", 9.0, pos, np.array([0, 1, 0], np.int32), [5, 3], [2.0, 1.7], 4, n_g,
                                  [seed], rotations="random")


def _angles(v):
    r = np.linalg.norm(v, axis=-1)
    return np.arccos(np.clip(v[..., 2] / r, -1, 1)), np.arctan2(v[..., 1], v[..., 0])


# ------------------------------------------------------------------------------- T matrices

@pytest.mark.parametrize("cfg", [0, "mixed"])
def test_tmat_hermitian_and_blocks(oracle_lib, cfg):
    cell = synthcells.config(0) if cfg == 0 else _mixed()
    for ty in range(cell.n_types):
        T = oracle_lib.tmat(cell, ty)
        nl = (cell.lmax[ty] + 1) ** 2
        assert T.shape == (2 * nl, 2 * nl)
        assert np.abs(T - T.conj().T).max() < 1e-15 * max(1.0, np.abs(T).max())
        assert np.abs(T.imag).max() == 0.0              # real under the reality rule of the inputs
        tab, tba = T[:nl, nl:], T[nl:, :nl]
        assert np.abs(tba - tab.conj().T).max() < 1e-15   # T^BA = (T^AB)^H (section 4.4)


def test_tmat_spherical_only(oracle_lib):
    cell = _mixed()
    for arr in (cell.i_uu, cell.i_ud, cell.i_du, cell.i_dd):
        arr[...] = 0.0
    for ty in range(cell.n_types):
        T = oracle_lib.tmat(cell, ty)
        lm = cell.lmax[ty]
        nl = (lm + 1) ** 2
        ls = np.repeat(np.arange(lm + 1), 2 * np.arange(lm + 1) + 1)
        el, un = cell.e_l[ty][ls], cell.ud_norm2[ty][ls]
        ref = np.zeros((2 * nl, 2 * nl))
        ref[:nl, :nl] = np.diag(el)
        ref[nl:, nl:] = np.diag(el * un)
        ref[:nl, nl:] = 0.5 * np.eye(nl)
        ref[nl:, :nl] = 0.5 * np.eye(nl)
        assert np.abs(T - ref).max() == 0.0


def test_tmat_literal_vs_symmetric(oracle_lib):
    cell = _mixed()
    for ty in range(cell.n_types):
        ts = oracle_lib.tmat(cell, ty)
        tl = oracle_lib.tmat(cell, ty, literal=True)
        nl = ts.shape[0] // 2
        d = tl - ts
        ref = np.zeros_like(d)
        ref[:nl, nl:] = 0.5 * np.eye(nl)
        ref[nl:, :nl] = -0.5 * np.eye(nl)
        assert np.abs(d - ref).max() < 1e-15
        assert np.abs(0.5 * (tl + tl.conj().T) - ts).max() < 1e-15


def _sphere_quadrature(n_theta, n_phi):
    z, w = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    Z, P = np.meshgrid(z, ph, indexing="ij")
    W = np.outer(w, np.full(n_phi, 2 * np.pi / n_phi))
    return np.arccos(Z).reshape(-1), P.reshape(-1), W.reshape(-1)


def test_tmat_by_angular_quadrature(oracle_lib):
    """T^[XY]_{L'L} - diagonal = sum_{L''} I^{xy}_{l'l L''} int conj(Y_L') Y_L'' Y_L, with the
    angular integral done by product quadrature over scipy's Y (no Gaunt formula)."""
    cell = _mixed()
    th, ph, w = _sphere_quadrature(12, 24)
    for ty in range(cell.n_types):
        lm, lp = int(cell.lmax[ty]), cell.lpot
        nl = (lm + 1) ** 2
        Y = np.array([sph_harm_y(l, m, th, ph) for l in range(lm + 1) for m in range(-l, l + 1)])
        Yp = np.array([sph_harm_y(l, m, th, ph) for l in range(lp + 1) for m in range(-l, l + 1)])
        ls = np.repeat(np.arange(lm + 1), 2 * np.arange(lm + 1) + 1)
        # V_{l'l}(Omega) = sum_L'' I_{l'l L''} Y_L''(Omega)
        T = oracle_lib.tmat(cell, ty)
        for blk, arr in enumerate((cell.i_uu, cell.i_ud, cell.i_du, cell.i_dd)):
            V = np.einsum("abq,qo->abo", arr[ty][: lm + 1, : lm + 1], Yp)
            Vfull = V[ls][:, ls]                                            # (nl, nl, npts)
            ref = np.einsum("po,pqo,qo,o->pq", Y.conj(), Vfull, Y, w)
            r0 = 0 if blk in (0, 1) else nl
            c0 = 0 if blk in (0, 2) else nl
            got = T[r0:r0 + nl, c0:c0 + nl]
            off = ~np.eye(nl, dtype=bool)
            assert np.abs(got[off] - ref[off]).max() < 1e-14
            dref = np.diag(ref).real + {0: cell.e_l[ty][ls], 1: 0.5, 2: 0.5,
                                        3: cell.e_l[ty][ls] * cell.ud_norm2[ty][ls]}[blk]
            assert np.abs(np.diag(T[r0:r0 + nl, c0:c0 + nl]) - dref).max() < 1e-14


# ------------------------------------------------------------------------------- coefficients

@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_coeffs_matching_conditions(oracle_lib, which):
    """A u(R) + B udot(R) and A u'(R) + B udot'(R) equal the value and radial derivative of the
    plane wave's l-component at the sphere (appendix A.1, the C^1 matching condition)."""
    cell = synthcells.config(0) if which == "c0" else _mixed()
    A, B = oracle_lib.coeffs(cell, 0)
    K = cell.kpts[0] + cell.gvecs[0]
    kn = np.linalg.norm(K, axis=1)
    off = 0
    for a in range(cell.n_atoms):
        ty = cell.atom_type[a]
        lm, R = cell.lmax[ty], cell.rmt[ty]
        th, ph = _angles((cell.rot[a] @ (K / kn[:, None]).T).T)
        phase = np.exp(1j * K @ cell.pos[a])
        for l in range(lm + 1):
            jl, djl = spherical_jn(l, kn * R), spherical_jn(l, kn * R, derivative=True)
            for m in range(-l, l + 1):
                row = off + l * l + l + m
                pre = 4 * np.pi / np.sqrt(cell.omega) * (1j ** l) * phase * np.conj(sph_harm_y(l, m, th, ph))
                v = A[row] * cell.u[ty, l] + B[row] * cell.ud[ty, l]
                d = A[row] * cell.du[ty, l] + B[row] * cell.dud[ty, l]
                assert np.abs(v - pre * jl).max() < 1e-14
                assert np.abs(d - pre * kn * djl).max() < 1e-14
        off += (lm + 1) ** 2


def test_coeffs_plane_wave_continuity(oracle_lib):
    """With a large l_max the muffin-tin function sum_L [A u + B udot] Y_L(R_a rhat) on the sphere
    reproduces the interstitial plane wave Omega^-1/2 exp(i K.(x_a + R rhat)) (eq. basis_function),
    and its radial derivative reproduces i (K.rhat) times it."""
    lm = 22
    cell = synthcells.custom_cell("big_l", 10.0, np.array([[1.0, 2.0, 3.0]]), np.array([0], np.int32), [lm], [1.3],
                                  2, 25, [21], rotations="random")
    A, B = oracle_lib.coeffs(cell, 0)
    K = cell.kpts[0] + cell.gvecs[0]
    rng = np.random.default_rng(3)
    rh = rng.standard_normal((40, 3))
    rh /= np.linalg.norm(rh, axis=1)[:, None]
    R = cell.rmt[0]
    Ra = cell.rot[0]
    th, ph = _angles((Ra @ rh.T).T)
    Y = np.array([sph_harm_y(l, m, th, ph) for l in range(lm + 1) for m in range(-l, l + 1)])   # (NL, npts)
    ls = np.repeat(np.arange(lm + 1), 2 * np.arange(lm + 1) + 1)
    val = (A * cell.u[0][ls][:, None] + B * cell.ud[0][ls][:, None]).T @ Y            # (n_g, npts)
    der = (A * cell.du[0][ls][:, None] + B * cell.dud[0][ls][:, None]).T @ Y
    pw = np.exp(1j * K @ (cell.pos[0][:, None] + R * rh.T)) / np.sqrt(cell.omega)
    assert np.abs(val - pw).max() < 1e-12
    assert np.abs(der - 1j * (K @ rh.T) * pw).max() < 1e-12


def test_coeffs_gamma_point(oracle_lib):
    """K_t = 0 (k = 0, G = 0): only l = 0 survives, the direction is irrelevant."""
    cell = synthcells.custom_cell("gamma", 8.0, np.array([[0.5, 1.0, 2.0]]), np.array([0], np.int32), [4], [2.0], 2, 7,
                                  [5], kpts=np.zeros((1, 3)))
    A, B = oracle_lib.coeffs(cell, 0)
    assert np.all(np.isfinite(A)) and np.all(np.isfinite(B))
    t0 = int(np.argmin(np.linalg.norm(cell.gvecs[0], axis=1)))
    assert np.linalg.norm(cell.gvecs[0][t0]) == 0.0
    assert np.abs(A[1:, t0]).max() == 0.0 and np.abs(B[1:, t0]).max() == 0.0
    W = cell.ud[0, 0] * cell.du[0, 0] - cell.u[0, 0] * cell.dud[0, 0]
    pre = 4 * np.pi / (W * np.sqrt(cell.omega)) / np.sqrt(4 * np.pi)
    assert abs(A[0, t0] - pre * (-cell.dud[0, 0])) < 1e-15
    assert abs(B[0, t0] - pre * cell.du[0, 0]) < 1e-15


# ------------------------------------------------------------------------------- S and H

def _full(oracle_lib, cell, ik=0):
    return oracle_lib.hs_full(cell, ik)


@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_hs_hermitian_psd_rank(oracle_lib, which):
    cell = synthcells.config(0) if which == "c0" else _mixed(n_g=150)
    H, S = _full(oracle_lib, cell)
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    assert np.abs(S - S.conj().T).max() < 1e-14 * np.abs(S).max()
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > -1e-13 * ev.max()
    k2 = 2 * cell.k_rows()
    n = cell.n_g(0)
    if n > k2:                                            # rank(S_MT) <= 2K
        assert np.sort(ev)[n - k2 - 1] < 1e-12 * ev.max()


def _legendre_S(cell, ik=0):
    """S from FLEUR's m-summed form (section 3.1), prefactor 4 pi / Omega (the printed
    (4 pi)^2 / Omega overcounts by the 1/(4 pi) of the addition theorem)."""
    K = cell.kpts[ik] + cell.gvecs[ik]
    kn = np.linalg.norm(K, axis=1)
    kh = K / kn[:, None]
    cosg = np.clip(kh @ kh.T, -1, 1)
    S = np.zeros((len(kn), len(kn)), complex)
    for a in range(cell.n_atoms):
        ty = cell.atom_type[a]
        R = cell.rmt[ty]
        ph = np.exp(1j * (K @ cell.pos[a]))
        pm = np.conj(ph)[:, None] * ph[None, :]
        for l in range(cell.lmax[ty] + 1):
            jl, djl = spherical_jn(l, kn * R), spherical_jn(l, kn * R, derivative=True)
            W = cell.ud[ty, l] * cell.du[ty, l] - cell.u[ty, l] * cell.dud[ty, l]
            fa = cell.ud[ty, l] * kn * djl - cell.dud[ty, l] * jl
            fb = -cell.u[ty, l] * kn * djl + cell.du[ty, l] * jl
            S += 4 * np.pi / cell.omega * pm * (2 * l + 1) * eval_legendre(l, cosg) * (
                np.outer(fa, fa) + cell.ud_norm2[ty, l] * np.outer(fb, fb)) / W ** 2
    return S


@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_S_legendre_closed_form(oracle_lib, which):
    cell = synthcells.config(0) if which == "c0" else _mixed(n_g=150)
    H, S = _full(oracle_lib, cell)
    Sl = _legendre_S(cell)
    assert np.abs(S - Sl).max() < 1e-13 * np.abs(S).max()


def test_S_rotation_invariance(oracle_lib):
    cell = _mixed(n_g=120)
    _, S1 = _full(oracle_lib, cell)
    cell.rot[:] = np.eye(3)
    _, S2 = _full(oracle_lib, cell)
    assert np.abs(S1 - S2).max() < 1e-13 * np.abs(S1).max()


def test_H_spherical_closed_form(oracle_lib):
    """With I = 0 and E_l = E for all l: H = E S + (A^H B + B^H A)/2."""
    cell = _mixed(n_g=120)
    for arr in (cell.i_uu, cell.i_ud, cell.i_du, cell.i_dd):
        arr[...] = 0.0
    cell.e_l[...] = -0.37
    H, S = _full(oracle_lib, cell)
    A, B = oracle_lib.coeffs(cell, 0)
    ref = -0.37 * S + 0.5 * (A.conj().T @ B + B.conj().T @ A)
    assert np.abs(H - ref).max() < 1e-13 * np.abs(H).max()


def test_H_literal_hermitian_part(oracle_lib):
    cell = _mixed(n_g=100)
    H, _ = oracle_lib.hs_full(cell, 0)
    Hl, _ = oracle_lib.hs_full(cell, 0, literal=True)
    assert np.abs(Hl - Hl.conj().T).max() > 1e-3 * np.abs(H).max()      # the printed form is not Hermitian
    assert np.abs(0.5 * (Hl + Hl.conj().T) - H).max() < 1e-13 * np.abs(H).max()


def test_H_linear_in_potential(oracle_lib):
    cell = _mixed(n_g=80)
    H1, _ = _full(oracle_lib, cell)
    for arr in (cell.i_uu, cell.i_ud, cell.i_du, cell.i_dd):
        arr *= 2.5
    H2, _ = _full(oracle_lib, cell)
    for arr in (cell.i_uu, cell.i_ud, cell.i_du, cell.i_dd):
        arr[...] = 0.0
    H0, _ = _full(oracle_lib, cell)
    assert np.abs((H2 - H0) - 2.5 * (H1 - H0)).max() < 1e-13 * np.abs(H1).max()


@pytest.mark.parametrize("seed", [11, 12])
def test_H_brute_force_angular_quadrature(oracle_lib, seed):
    """H written out from eq. h_expanded_basis: per atom the muffin-tin functions
    F^x_{l}(t, Omega) = sum_m C^x_{lm}(t) Y_lm(Omega) (C^A = A, C^B = B) are combined with
    V^{xy}_{l'l}(Omega) = sum_L'' I^{xy}_{l'lL''} Y_L''(Omega) and integrated over the sphere by
    quadrature, plus the spherical Hamiltonian <u|H|u> = E, <u|H|udot> = <udot|H|u> = 1/2
    (Hermitian part), <udot|H|udot> = E ||udot||^2."""
    cell = _tiny(seed=seed)
    H, S = _full(oracle_lib, cell)
    A, B = oracle_lib.coeffs(cell, 0)
    th, ph, w = _sphere_quadrature(10, 20)
    n = cell.n_g(0)
    ref = np.zeros((n, n), complex)
    off = 0
    for a in range(cell.n_atoms):
        ty = cell.atom_type[a]
        lm = int(cell.lmax[ty])
        nl = (lm + 1) ** 2
        Y = np.array([sph_harm_y(l, m, th, ph) for l in range(lm + 1) for m in range(-l, l + 1)])
        Yp = np.array([sph_harm_y(l, m, th, ph) for l in range(cell.lpot + 1) for m in range(-l, l + 1)])
        ls = np.repeat(np.arange(lm + 1), 2 * np.arange(lm + 1) + 1)
        C = {"A": A[off:off + nl], "B": B[off:off + nl]}
        F = {x: np.stack([(C[x][ls == l][:, :, None] * Y[ls == l][:, None, :]).sum(0) for l in range(lm + 1)])
             for x in C}                                    # (l, t, Omega)
        ints = {("A", "A"): cell.i_uu, ("A", "B"): cell.i_ud, ("B", "A"): cell.i_du, ("B", "B"): cell.i_dd}
        for (x, y), arr in ints.items():
            V = np.einsum("abq,qo->abo", arr[ty][: lm + 1, : lm + 1], Yp)
            ref += np.einsum("pso,pqo,qto,o->st", F[x].conj(), V, F[y], w)
        el, un = cell.e_l[ty][ls], cell.ud_norm2[ty][ls]
        a_, b_ = C["A"], C["B"]
        ref += (a_.conj().T * el) @ a_ + 0.5 * a_.conj().T @ b_ + 0.5 * b_.conj().T @ a_ + (b_.conj().T * (el * un)) @ b_
        off += nl
    assert np.abs(H - ref).max() < 1e-13 * np.abs(H).max()


def test_sampled_equals_full(oracle_lib):
    cell = _mixed(n_g=140)
    H, S = _full(oracle_lib, cell)
    rows = np.array([0, 5, 17, 88, 139])
    cols = np.array([3, 17, 100, 139])
    Hs, Ss = oracle_lib.hs_sampled(cell, 0, rows, cols)
    assert np.abs(Hs - H[np.ix_(rows, cols)]).max() < 1e-14 * np.abs(H).max()
    assert np.abs(Ss - S[np.ix_(rows, cols)]).max() < 1e-14 * np.abs(S).max()


# ------------------------------------------------------------------ structured T (section 3.1)

def _with_spherical_slot(cell, seed=5):
    """Give the l'' = 0 slot nonzero values (the generator leaves it zero) with the symmetries
    of the integrals: I^uu, I^dd symmetric in (l', l), I^du = (I^ud)^T."""
    rng = np.random.default_rng(seed)
    for ty in range(cell.n_types):
        for lp in range(cell.lstride):
            for l in range(lp, cell.lstride):
                for arr in (cell.i_uu, cell.i_dd):
                    v = rng.normal(0, 0.1)
                    arr[ty, lp, l, 0] = arr[ty, l, lp, 0] = v
                v = rng.normal(0, 0.1)
                cell.i_ud[ty, lp, l, 0] = cell.i_du[ty, l, lp, 0] = v
                v = rng.normal(0, 0.1)
                cell.i_ud[ty, l, lp, 0] = cell.i_du[ty, lp, l, 0] = v
    return cell


def test_tmat_structured_no_cut_is_full(oracle_lib):
    cell = _mixed()
    for ty in range(cell.n_types):
        full = oracle_lib.tmat(cell, ty)
        for lns in (int(cell.lmax[ty]), 12):
            assert np.array_equal(oracle_lib.tmat(cell, ty, lnonsph=lns), full)


@pytest.mark.parametrize("lns", [0, 1, 2])
def test_tmat_structured_blocks(oracle_lib, lns):
    """Dense block l', l <= lns equal to the full T; outside it nothing but the diagonal, which
    equals the T of the same potential with every l'' >= 1 integral removed (Fig. Tmat_structure)."""
    cell = _with_spherical_slot(_mixed())
    sph = _with_spherical_slot(_mixed())
    for arr in (sph.i_uu, sph.i_ud, sph.i_du, sph.i_dd):
        arr[..., 1:] = 0.0
    for ty in range(cell.n_types):
        lm = int(cell.lmax[ty])
        nl = (lm + 1) ** 2
        nd = (lns + 1) ** 2
        full = oracle_lib.tmat(cell, ty)
        st = oracle_lib.tmat(cell, ty, lnonsph=lns)
        ts = oracle_lib.tmat(sph, ty)
        inside = np.zeros(nl, bool)
        inside[:nd] = True
        inside2 = np.concatenate([inside, inside])
        dense = inside2[:, None] & inside2[None, :]
        assert np.array_equal(st[dense], full[dense])
        L = np.tile(np.arange(nl), 2)
        same_L = L[:, None] == L[None, :]
        outside = ~dense
        assert np.all(st[outside & ~same_L] == 0.0)
        assert np.array_equal(st[outside & same_L], ts[outside & same_L])
        assert np.any(full[outside & ~same_L] != 0.0)          # the cut removes something


def test_H_structured_T_plumbing(oracle_lib):
    """hs_full with lnonsph equals the definition evaluated with the structured T."""
    cell = _with_spherical_slot(_mixed(n_g=70))
    H, S = oracle_lib.hs_full(cell, 0, lnonsph=2)
    T = oracle_lib.tmat_all(cell, lnonsph=2)
    A, B = oracle_lib.coeffs(cell, 0)
    H2, S2 = oracle_lib.hs_block(cell, T, A, B, A, B)
    assert np.array_equal(H, H2) and np.array_equal(S, S2)
    Hf, Sf = oracle_lib.hs_full(cell, 0)
    assert np.array_equal(S, Sf)                                 # S does not involve T
    assert np.abs(H - Hf).max() > 1e-6 * np.abs(Hf).max()
