"""Seeded synthetic FLAPW cells: the inputs that both the GPU path and the oracle consume.

This module holds no part of the method's arithmetic (no coefficients, no T matrices,
no H or S).  It only draws inputs: a crystal cell, atoms with positions and rotations,
per-type radial boundary values, non-spherical radial integrals, k-points and, per
k-point, the list of reciprocal lattice vectors G_t that form the basis.

Problem statement being fed (the paper's section 2.2 and appendix A):
  * basis functions are labelled by K_t = k + G_t with |K_t| <= K_max (section 2.2);
  * per atom a: position x_a, rotation R_a, type (appendix A.1);
  * per type and l: u(R), u'(R), udot(R), udot'(R) at the muffin-tin radius R,
    ||udot_l||^2 and the energy parameter E_l (eqs. def_a_tensor, def_b_tensor,
    def_overlap, t_matrices);
  * per type: non-spherical radial integrals I^{(x,y)}_{l',l,L''} (eq. nonsph_integrals).

Conventions (readings of points the paper leaves open):
  * atomic units; reciprocal vectors b_i = 2 pi (A^-T)_i; Omega = |det A|;
  * the basis for one k-point is the N_G shortest |k+G| (ties broken by the integer
    triple n lexicographically), which is the set |K_t| <= K_max for K_max between the
    N_G-th and the (N_G+1)-th norm;
  * I arrays are indexed [type][l'][l][L''] with L'' = l''^2 + l'' + m'' and the bra
    function first; I^{uu}, I^{udot udot} symmetric in (l', l); every I obeys the
    reality rule I_{(l'',-m)} = (-1)^m I_{(l'',m)}; the l''=0 slot is zero (it belongs
    to the spherical Hamiltonian); I^{udot u}_{l',l,L''} = I^{u udot}_{l,l',L''};
  * (u, u', udot, udot') of one (type, l) are redrawn until |W| >= 0.05 with
    W = udot u' - u udot'.

The five named workloads follow the paper's sizes (N_G ~ 50-80 per atom, l_max <= 10,
section 2.3): a 2-atom cell with N_G = 300, a 64-atom rock-salt supercell with N_G = 3000, a
256-atom fcc cell with l_max = 10 and N_G = 6000, a 32-atom cell with 64 k-points of uneven
N_G in [2000, 4500], and a 512-atom cell with 4 k-points of N_G in [11000, 12500].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = ["Cell", "config", "config_separated", "custom_cell", "kset", "random_contraction_inputs", "radial_meshes", "RadialMeshes",
           "CONFIG_NAMES"]

CONFIG_NAMES = ["c0_small", "c1_realistic", "c2_precision", "c3_batched", "c4_scale"]


@dataclass
class Cell:
    name: str
    lattice: np.ndarray            # (3,3) rows are lattice vectors (bohr)
    omega: float                   # cell volume (bohr^3)
    pos: np.ndarray                # (n_atoms,3) Cartesian positions (bohr)
    rot: np.ndarray                # (n_atoms,3,3) row-major orthogonal matrices
    atom_type: np.ndarray          # (n_atoms,) int32
    lmax: np.ndarray               # (n_types,) int32
    rmt: np.ndarray                # (n_types,) muffin-tin radii (bohr)
    u: np.ndarray                  # (n_types, lstride) u_l(R)
    du: np.ndarray                 # u_l'(R)
    ud: np.ndarray                 # udot_l(R)
    dud: np.ndarray                # udot_l'(R)
    ud_norm2: np.ndarray           # ||udot_l||^2
    e_l: np.ndarray                # E_l
    lpot: int                      # l''_max of the non-spherical potential
    i_uu: np.ndarray               # (n_types, lstride, lstride, (lpot+1)^2)
    i_ud: np.ndarray               # I^{(u, udot)}
    i_du: np.ndarray               # I^{(udot, u)}
    i_dd: np.ndarray               # I^{(udot, udot)}
    kpts: np.ndarray               # (n_k,3) Cartesian k (bohr^-1)
    gvecs: List[np.ndarray] = field(default_factory=list)   # per k: (n_g,3) Cartesian G
    gint: List[np.ndarray] = field(default_factory=list)    # per k: (n_g,3) integer triples

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_types(self) -> int:
        return int(self.lmax.shape[0])

    @property
    def lstride(self) -> int:
        return int(self.u.shape[1])

    @property
    def n_k(self) -> int:
        return int(self.kpts.shape[0])

    def n_g(self, ik: int) -> int:
        return int(self.gvecs[ik].shape[0])

    def nl_atom(self) -> np.ndarray:
        return ((self.lmax[self.atom_type] + 1) ** 2).astype(np.int64)

    def k_rows(self) -> int:
        """K = sum over atoms of (l_max(type)+1)^2 (rows of the stacked A or B)."""
        return int(self.nl_atom().sum())

    def reciprocal(self) -> np.ndarray:
        return 2.0 * np.pi * np.linalg.inv(self.lattice).T

    def flops_per_k(self, ik: int) -> float:
        """Algorithmic flops of one k-point: S and H upper triangles (8 K N(N+1) each,
        a complex multiply-add counted as 8 real flops) plus the per-atom panels T_a P_a
        (32 N sum_a N_La^2)."""
        n = float(self.n_g(ik))
        k = float(self.k_rows())
        nl = self.nl_atom().astype(np.float64)
        return 16.0 * k * n * (n + 1.0) + 32.0 * n * float((nl * nl).sum())


# ----------------------------------------------------------------------------------------
# building blocks


def _rng(tag) -> np.random.Generator:
    return np.random.default_rng(tag)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def kset(lattice: np.ndarray, k_cart: np.ndarray, n_g: int):
    """The n_g vectors G = n1 b1 + n2 b2 + n3 b3 with the smallest |k+G|.

    Returns (G Cartesian (n_g,3), n integer (n_g,3), K_max) where K_max is the midpoint
    between the n_g-th and (n_g+1)-th norm, so the list is exactly {G : |k+G| <= K_max}.
    """
    omega = abs(np.linalg.det(lattice))
    b = 2.0 * np.pi * np.linalg.inv(lattice).T
    kmax_est = (6.0 * np.pi ** 2 * (n_g + 1) / omega) ** (1.0 / 3.0)
    radius = 1.35 * kmax_est + np.linalg.norm(k_cart) + 1e-9
    while True:
        nmax = [int(np.ceil(radius * np.linalg.norm(lattice[i]) / (2.0 * np.pi))) + 1 for i in range(3)]
        r = [np.arange(-m, m + 1) for m in nmax]
        n = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
        g = n @ b
        norm = np.linalg.norm(g + k_cart[None, :], axis=1)
        inside = norm <= radius
        if inside.sum() > n_g:
            break
        radius *= 1.3
    n, g, norm = n[inside], g[inside], norm[inside]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0], norm))
    sel = order[: n_g]
    kmax = 0.5 * (norm[order[n_g - 1]] + norm[order[n_g]])
    return g[sel].copy(), n[sel].astype(np.int32), float(kmax)


def _radial(rng: np.random.Generator, lmax: np.ndarray, lstride: int):
    nt = lmax.shape[0]
    u = np.zeros((nt, lstride)); du = np.zeros_like(u); ud = np.zeros_like(u); dud = np.zeros_like(u)
    udn = np.zeros_like(u); el = np.zeros_like(u)
    for t in range(nt):
        for l in range(lmax[t] + 1):
            while True:
                a, b, c, d = rng.uniform(0.1, 1.0, size=4)
                if abs(c * b - a * d) >= 0.05:
                    break
            u[t, l], du[t, l], ud[t, l], dud[t, l] = a, b, c, d
            udn[t, l] = rng.uniform(0.01, 0.1)
            el[t, l] = rng.uniform(-1.0, 1.0)
    return u, du, ud, dud, udn, el


def _reality(x: np.ndarray, lpot: int) -> np.ndarray:
    """Impose I_{(l'',-m)} = (-1)^m I_{(l'',m)} on the last axis; zero the l''=0 slot."""
    x = x.copy()
    x[..., 0] = 0.0
    for lpp in range(1, lpot + 1):
        for m in range(1, lpp + 1):
            x[..., lpp * lpp + lpp - m] = (-1) ** m * x[..., lpp * lpp + lpp + m]
    return x


def _integrals(rng: np.random.Generator, lmax: np.ndarray, lstride: int, lpot: int, sigma: float = 0.1):
    nt = lmax.shape[0]
    nlp = (lpot + 1) ** 2
    i_uu = np.zeros((nt, lstride, lstride, nlp)); i_dd = np.zeros_like(i_uu); i_ud = np.zeros_like(i_uu)
    for t in range(nt):
        n = lmax[t] + 1
        for arr, sym in ((i_uu, True), (i_dd, True), (i_ud, False)):
            x = rng.normal(0.0, sigma, size=(n, n, nlp))
            if sym:
                iu0, iu1 = np.triu_indices(n)
                y = np.zeros_like(x)
                y[iu0, iu1, :] = x[iu0, iu1, :]
                y[iu1, iu0, :] = x[iu0, iu1, :]
                x = y
            arr[t, :n, :n, :] = _reality(x, lpot)
    i_du = i_ud.transpose(0, 2, 1, 3).copy()
    return i_uu, i_ud, i_du, i_dd


def _fcc_sites(ncell: int, side: float) -> np.ndarray:
    base = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    out = []
    for i in range(ncell):
        for j in range(ncell):
            for k in range(ncell):
                out.append((base + np.array([i, j, k])) * side)
    return np.concatenate(out, axis=0)


def _rocksalt_sites(ncell: int, side: float):
    a = _fcc_sites(ncell, side)
    b = a + np.array([0.5 * side, 0.0, 0.0])
    return a, b


def _kpoints(rng: np.random.Generator, lattice: np.ndarray, n_k: int) -> np.ndarray:
    frac = rng.uniform(-0.5, 0.5, size=(n_k, 3))
    return frac @ (2.0 * np.pi * np.linalg.inv(lattice).T)


def custom_cell(name: str, a: float, pos: np.ndarray, atom_type: np.ndarray, lmax_t, rmt_t, lpot: int,
                n_g, seed, rotations: str = "identity", kpts: Optional[np.ndarray] = None) -> Cell:
    """A cubic cell of side a with the given atoms; per-type radial data and integrals are
    drawn from the seeded generator.  n_g is an int or a list (one entry per k-point)."""
    rng = _rng(seed)
    lattice = np.eye(3) * a
    lmax = np.asarray(lmax_t, dtype=np.int32)
    rmt = np.asarray(rmt_t, dtype=np.float64)
    lstride = int(lmax.max()) + 1
    n_atoms = pos.shape[0]
    if rotations == "identity":
        rot = np.tile(np.eye(3), (n_atoms, 1, 1))
    else:
        rot = np.stack([random_rotation(rng) for _ in range(n_atoms)])
    u, du, ud, dud, udn, el = _radial(rng, lmax, lstride)
    i_uu, i_ud, i_du, i_dd = _integrals(rng, lmax, lstride, lpot)
    ngs = [int(n_g)] if np.isscalar(n_g) else [int(x) for x in n_g]
    if kpts is None:
        kpts = _kpoints(rng, lattice, len(ngs))
    gv, gi = [], []
    for ik in range(kpts.shape[0]):
        g, n, _ = kset(lattice, kpts[ik], ngs[ik])
        gv.append(g); gi.append(n)
    return Cell(name=name, lattice=lattice, omega=float(abs(np.linalg.det(lattice))), pos=np.asarray(pos, float),
                rot=rot, atom_type=np.asarray(atom_type, dtype=np.int32), lmax=lmax, rmt=rmt, u=u, du=du, ud=ud,
                dud=dud, ud_norm2=udn, e_l=el, lpot=int(lpot), i_uu=i_uu, i_ud=i_ud, i_du=i_du, i_dd=i_dd,
                kpts=np.asarray(kpts, float), gvecs=gv, gint=gi)


def config(i: int, n_k: Optional[int] = None) -> Cell:
    """The five named workloads (0..4).  n_k truncates the k-point list (for tests)."""
    seed = [1602, 6589, i]
    rng = _rng(seed + [99])
    if i == 0:
        a = 8.0
        pos = rng.uniform(0.0, 1.0, size=(2, 3)) * a
        cell = custom_cell(CONFIG_NAMES[0], a, pos, np.zeros(2, np.int32), [6], [2.0], 4, 300, seed)
    elif i == 1:
        sa, sb = _rocksalt_sites(2, 10.0)
        pos = np.concatenate([sa, sb])
        typ = np.concatenate([np.zeros(len(sa), np.int32), np.ones(len(sb), np.int32)])
        cell = custom_cell(CONFIG_NAMES[1], 20.0, pos, typ, [8, 8], [2.2, 2.4], 6, 3000, seed)
    elif i == 2:
        pos = _fcc_sites(4, 8.0)
        typ = rng.permutation(np.repeat(np.arange(4, dtype=np.int32), 64))
        cell = custom_cell(CONFIG_NAMES[2], 32.0, pos, typ, [10] * 4, [2.0, 2.2, 2.4, 2.6], 8, 6000, seed,
                           rotations="random")
    elif i == 3:
        pos = _fcc_sites(2, 10.0)
        typ = (np.arange(32) % 2).astype(np.int32)
        ngs = rng.integers(2000, 4501, size=64)
        cell = custom_cell(CONFIG_NAMES[3], 20.0, pos, typ, [8, 8], [2.2, 2.4], 6,
                           list(ngs[: (n_k or 64)]), seed)
    elif i == 4:
        sa, sb = _rocksalt_sites(4, 10.0)
        ta = rng.integers(0, 4, size=len(sa)).astype(np.int32)
        tb = rng.integers(4, 8, size=len(sb)).astype(np.int32)
        pos = np.concatenate([sa, sb])
        typ = np.concatenate([ta, tb])
        ngs = rng.integers(11000, 12501, size=4)
        cell = custom_cell(CONFIG_NAMES[4], 40.0, pos, typ, [10] * 8, [2.0 + 0.05 * t for t in range(8)], 8,
                           list(ngs[: (n_k or 4)]), seed, rotations="random")
    else:
        raise ValueError(f"unknown config {i}")
    return cell


def min_sphere_gap(cell: Cell) -> float:
    """Smallest distance between two muffin-tin spheres over the periodic images (negative when two
    overlap): min over atom pairs of |x_b - x_a| (minimum image) - R_a - R_b."""
    inv = np.linalg.inv(cell.lattice)
    R = cell.rmt[cell.atom_type]
    gap = np.inf
    for a in range(cell.n_atoms):
        d = cell.pos - cell.pos[a]
        f = d @ inv
        f -= np.round(f)
        dist = np.linalg.norm(f @ cell.lattice, axis=1)
        dist[a] = np.inf
        gap = min(gap, float(np.min(dist - R - R[a])))
    return gap


def config_separated(i: int, n_k: Optional[int] = None) -> Cell:
    """A named workload whose muffin-tin spheres do not overlap, as the interstitial region needs.
    Workloads 1-4 already qualify and are returned as they are; workload 0 (two atoms at random
    positions, whose spheres overlap) keeps its cell, type, l_max, radial data, k-point and basis,
    with its positions redrawn (seeded) until the spheres are at least 0.5 bohr apart."""
    cell = config(i, n_k)
    if i != 0:
        return cell
    rng = _rng([1602, 6589, 0, 7])
    while True:
        cell.pos = rng.uniform(0.0, 1.0, size=(cell.n_atoms, 3)) * cell.lattice[0, 0]
        if min_sphere_gap(cell) >= 0.5:
            return cell


def random_contraction_inputs(seed, k_rows: int, n_g: int):
    """Random stacked A_*, B_* (K x N complex128, column-major) for testing the
    contraction stage on inputs that are not coefficient-shaped."""
    rng = _rng(seed)
    a = rng.standard_normal((k_rows, n_g)) + 1j * rng.standard_normal((k_rows, n_g))
    b = rng.standard_normal((k_rows, n_g)) + 1j * rng.standard_normal((k_rows, n_g))
    return np.asfortranarray(a), np.asfortranarray(b)


@dataclass
class RadialMeshes:
    """Radial meshes and potentials of the atom types (inputs of the radial solve)."""
    n_r: int                       # points per mesh, r_i = r0 (R/r0)^(i/(n_r-1))
    r0: np.ndarray                 # (n_types,) first mesh point (bohr)
    rmt: np.ndarray                # (n_types,) muffin-tin radius (bohr)
    lmax: np.ndarray               # (n_types,) int32
    z: np.ndarray                  # (n_types,) nuclear charge used for v_sph
    e_l: np.ndarray                # (n_types, lstride) energy parameters (hartree)
    v_sph: np.ndarray              # (n_types, n_r) spherical potential (hartree)
    lpot: int
    v_lm: np.ndarray               # (n_types, (lpot+1)^2, n_r) non-spherical components


def radial_meshes(lmax, rmt, lpot: int, n_r: int = 1001, seed=0, lstride: Optional[int] = None,
                  r0=None) -> RadialMeshes:
    """Seeded synthetic muffin-tin potentials on logarithmic meshes (Hartree units).

    Per type: nuclear charge Z in 3..40; r0 in [1e-6, 1e-5]; the spherical potential of a nucleus
    inside a uniform neutralising sphere of radius R, -Z/r + Z (3R^2 - r^2)/(2R^3), plus a constant
    in [-0.3, 0.3]; E_l in [-0.5, 1.0].  Non-spherical components for l'' >= 1:
    v_{l'',m}(r) = a (r/R)^{l''} (1 + b r/R) with a ~ N(0, 0.2/l''), b in [-1, 1], drawn for
    m >= 0 and mirrored by v_{l'',-m} = (-1)^m v_{l'',m} (a real potential with real components);
    the l''=0 component is zero (it belongs to the spherical potential).  n_r - 1 must be a
    multiple of 4 (the solve steps over two mesh intervals and Simpson's rule over pairs of steps).
    r0, when given, replaces the drawn first mesh points (one value or one per type).
    """
    if (n_r - 1) % 4:
        raise ValueError("n_r - 1 must be a multiple of 4")
    lmax = np.asarray(lmax, dtype=np.int32)
    rmt = np.asarray(rmt, dtype=np.float64)
    nt = lmax.shape[0]
    ls = int(lstride or lmax.max() + 1)
    rng = _rng([7919, int(seed)])
    nlp = (lpot + 1) ** 2
    z = rng.integers(3, 41, size=nt).astype(np.float64)
    r0 = rng.uniform(1e-6, 1e-5, size=nt) if r0 is None else np.broadcast_to(np.asarray(r0, np.float64), (nt,)).copy()
    e_l = np.zeros((nt, ls))
    v_sph = np.zeros((nt, n_r))
    v_lm = np.zeros((nt, nlp, n_r))
    for t in range(nt):
        R = rmt[t]
        r = r0[t] * (R / r0[t]) ** (np.arange(n_r) / (n_r - 1))
        v_sph[t] = -z[t] / r + z[t] * (3 * R * R - r * r) / (2 * R ** 3) + rng.uniform(-0.3, 0.3)
        e_l[t, : lmax[t] + 1] = rng.uniform(-0.5, 1.0, size=lmax[t] + 1)
        x = r / R
        for lpp in range(1, lpot + 1):
            for m in range(0, lpp + 1):
                a, b = rng.normal(0.0, 0.2 / lpp), rng.uniform(-1.0, 1.0)
                comp = a * x ** lpp * (1.0 + b * x)
                v_lm[t, lpp * lpp + lpp + m] = comp
                if m:
                    v_lm[t, lpp * lpp + lpp - m] = (-1) ** m * comp
    return RadialMeshes(n_r, r0, rmt.copy(), lmax, z, e_l, v_sph, int(lpot), v_lm)
