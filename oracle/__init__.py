"""CPU FP64 oracle for FLAPW muffin-tin H and S generation -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1602_06589_amd``) and never imports it.

The arithmetic lives in ``flapw_oracle.c`` (plain loops, OpenMP over output columns);
this module only marshals numpy arrays through ctypes.  Functions:

  sph_bessel(lmax, x)          j_l(x), j_l'(x)                      appendix A.1
  ylm(lmax, v)                 Y_lm(v/|v|), Condon-Shortley          section 2.2
  wigner3j, gaunt              G_{L,L',L''} = int conj(Y_L') Y_L Y_L''  appendix A.2, eq. gaunt
  tmat(cell, type)             [[T^AA, T^AB], [T^BA, T^BB]]          appendix A.2, eq. t_matrices
  coeffs(cell, ik, cols)       A_*, B_* (K x n)                      appendix A.1, eqs. def_a/def_b
  hs_block(cell, ...)          blocks of H and S                     section 2.3, eqs. def_overlap,
                                                                     def_hamilton
  interstitial_block(cell, ..) interstitial blocks of H and S        section 2.3, eqs. basis_function
                                                                     (INT), HS_Mat
  eigh_generalized(H, S)       H c = eps S c                         section 2.3, eq. matrix_kohnsham
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flapw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the path of the library."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            L = ctypes.c_long
            lib.or_sph_bessel.argtypes = [I, D, P, P]
            lib.or_ylm.argtypes = [I, P, P]
            lib.or_wigner3j.argtypes = [I] * 6
            lib.or_wigner3j.restype = D
            lib.or_gaunt.argtypes = [I] * 6
            lib.or_gaunt.restype = D
            lib.or_tmat.argtypes = [I, I, I, P, P, P, P, P, P, I, I, P, I]
            lib.or_coeffs.argtypes = [I, P, P, P, D, I, P, P, P, P, P, P, P, I, P, P, P, L]
            lib.or_hs_block.argtypes = [I, P, P, I, P, P, I, I, L, I, P, P, L, I, P, P, L, P, P]
            lib.or_radial.argtypes = [I, D, D, P, I, D, P, P, P]
            lib.or_interstitial_block.argtypes = [I, P, P, P, D, D, P, I, P, I, P, P, P]
            lib.or_radial_integral.argtypes = [I, D, D, P, P, P]
            lib.or_radial_integral.restype = D
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def sph_bessel(lmax: int, x: float):
    j = np.zeros(lmax + 1)
    dj = np.zeros(lmax + 1)
    _load().or_sph_bessel(int(lmax), float(x), _p(j), _p(dj))
    return j, dj


def ylm(lmax: int, v) -> np.ndarray:
    y = np.zeros((lmax + 1) ** 2, dtype=np.complex128)
    vv = _c(v, np.float64)
    _load().or_ylm(int(lmax), _p(vv), _p(y))
    return y


def wigner3j(j1, j2, j3, m1, m2, m3) -> float:
    return _load().or_wigner3j(j1, j2, j3, m1, m2, m3)


def gaunt(l, m, lp, mp, lpp, mpp) -> float:
    """G_{L,L',L''} = int conj(Y_{l'm'}) Y_{lm} Y_{l''m''} dOmega."""
    return _load().or_gaunt(l, m, lp, mp, lpp, mpp)


def tmat(cell, ty: int, literal: bool = False, ldt: int | None = None, lnonsph: int = -1) -> np.ndarray:
    """T of one atom type as a (2NL x 2NL) complex array (bra rows, ket columns).  lnonsph >= 0:
    the structured T of section 3.1 (non-spherical terms only for l', l <= lnonsph)."""
    lm = int(cell.lmax[ty])
    nl = (lm + 1) ** 2
    ldt = ldt or 2 * nl
    t = np.zeros((2 * nl, ldt), dtype=np.complex128)     # column-major storage: t[col, row]
    ls = cell.lstride
    args = [_c(cell.i_uu[ty], np.float64), _c(cell.i_ud[ty], np.float64), _c(cell.i_du[ty], np.float64),
            _c(cell.i_dd[ty], np.float64)]
    el = _c(cell.e_l[ty], np.float64)
    un = _c(cell.ud_norm2[ty], np.float64)
    _load().or_tmat(lm, ls, int(cell.lpot), *[_p(a) for a in args], _p(el), _p(un), int(bool(literal)), int(lnonsph),
                      _p(t), ldt)
    return t[:, : 2 * nl].T.copy()


def tmat_all(cell, literal: bool = False, lnonsph: int = -1) -> np.ndarray:
    """All types, padded: (n_types, 2 NLmax, 2 NLmax), each type's matrix top-left."""
    nlmax = int((cell.lmax.max() + 1) ** 2)
    out = np.zeros((cell.n_types, 2 * nlmax, 2 * nlmax), dtype=np.complex128)
    for ty in range(cell.n_types):
        t = tmat(cell, ty, literal, lnonsph=lnonsph)
        out[ty, : t.shape[0], : t.shape[1]] = t
    return out


def coeffs(cell, ik: int, cols=None):
    """A_*, B_* for k-point ik, restricted to the basis columns `cols` (default: all).
    Returns two (K x n) complex arrays."""
    g = cell.gvecs[ik] if cols is None else cell.gvecs[ik][np.asarray(cols)]
    g = _c(g, np.float64)
    n = g.shape[0]
    k = cell.k_rows()
    A = np.zeros((n, k), dtype=np.complex128)            # column-major K x n
    B = np.zeros((n, k), dtype=np.complex128)
    _load().or_coeffs(cell.n_atoms, _p(_c(cell.atom_type, np.int32)), _p(_c(cell.pos, np.float64)),
                      _p(_c(cell.rot, np.float64)), float(cell.omega), cell.lstride, _p(_c(cell.lmax, np.int32)),
                      _p(_c(cell.rmt, np.float64)), _p(_c(cell.u, np.float64)), _p(_c(cell.du, np.float64)),
                      _p(_c(cell.ud, np.float64)), _p(_c(cell.dud, np.float64)), _p(_c(cell.kpts[ik], np.float64)),
                      n, _p(g), _p(A), _p(B), k)
    return A.T, B.T


def hs_block(cell, T, Al, Bl, Ar, Br):
    """H and S entries for bra columns (Al, Bl: K x nr) and ket columns (Ar, Br: K x nc).
    T is tmat_all(cell).  Returns (H, S) as (nr x nc) arrays."""
    k = cell.k_rows()
    nlmax = int((cell.lmax.max() + 1) ** 2)
    ldt = 2 * nlmax
    # column-major per type: element (row, col) at col * ldt + row
    Tc = np.ascontiguousarray(np.transpose(T, (0, 2, 1)), dtype=np.complex128)
    Alc = np.ascontiguousarray(np.asarray(Al).T, dtype=np.complex128)
    Blc = np.ascontiguousarray(np.asarray(Bl).T, dtype=np.complex128)
    Arc = np.ascontiguousarray(np.asarray(Ar).T, dtype=np.complex128)
    Brc = np.ascontiguousarray(np.asarray(Br).T, dtype=np.complex128)
    nr, nc = Alc.shape[0], Arc.shape[0]
    H = np.zeros((nc, nr), dtype=np.complex128)
    S = np.zeros((nc, nr), dtype=np.complex128)
    _load().or_hs_block(cell.n_atoms, _p(_c(cell.atom_type, np.int32)), _p(_c(cell.lmax, np.int32)), cell.lstride,
                        _p(_c(cell.ud_norm2, np.float64)), _p(Tc), ldt, nlmax, k, nr, _p(Alc), _p(Blc), k, nc,
                        _p(Arc), _p(Brc), k, _p(H), _p(S))
    return H.T, S.T


def hs_full(cell, ik: int, literal: bool = False, lnonsph: int = -1):
    """Full N x N H and S of one k-point (small problems only); lnonsph as in tmat."""
    T = tmat_all(cell, literal, lnonsph)
    A, B = coeffs(cell, ik)
    return hs_block(cell, T, A, B, A, B)


def hs_sampled(cell, ik: int, rows, cols, T=None):
    """H[rows][:, cols] and S[rows][:, cols] computed entry by entry from the coefficients of
    just those basis functions (cheap at any size)."""
    T = tmat_all(cell) if T is None else T
    Al, Bl = coeffs(cell, ik, rows)
    Ar, Br = coeffs(cell, ik, cols)
    return hs_block(cell, T, Al, Bl, Ar, Br)


def interstitial_block(cell, ik: int, rows=None, cols=None, v_int: float = 0.0):
    """Interstitial H and S (plane waves integrated over the cell minus the muffin-tin spheres) for
    the basis functions `rows` (bra) and `cols` (ket) of k-point ik (default: all).  Returns (H, S)
    as (nr x nc) arrays."""
    g = cell.gvecs[ik]
    gr = _c(g if rows is None else g[np.asarray(rows)], np.float64)
    gc = _c(g if cols is None else g[np.asarray(cols)], np.float64)
    nr, nc = gr.shape[0], gc.shape[0]
    H = np.zeros((nc, nr), dtype=np.complex128)
    S = np.zeros((nc, nr), dtype=np.complex128)
    _load().or_interstitial_block(cell.n_atoms, _p(_c(cell.atom_type, np.int32)), _p(_c(cell.rmt, np.float64)),
                                  _p(_c(cell.pos, np.float64)), float(cell.omega), float(v_int),
                                  _p(_c(cell.kpts[ik], np.float64)), nr, _p(gr), nc, _p(gc), _p(H), _p(S))
    return H.T, S.T


def hs_total(cell, ik: int, v_int: float = 0.0, lnonsph: int = -1):
    """Full N x N H and S of one k-point including the interstitial region (muffin-tin part of
    hs_full plus interstitial_block); small problems only."""
    Hm, Sm = hs_full(cell, ik, lnonsph=lnonsph)
    Hi, Si = interstitial_block(cell, ik, v_int=v_int)
    return Hm + Hi, Sm + Si


def eigh_generalized(H, S):
    """Eigenvalues (ascending) and S-orthonormal eigenvectors of H c = eps S c (section 2.3, eq.
    matrix_kohnsham) for Hermitian H and positive definite S, by the library routine
    scipy.linalg.eigh (full matrices, both triangles given)."""
    import scipy.linalg
    return scipy.linalg.eigh(H, S)


# ----------------------------------------------------------------------------- radial functions

def radial_mesh(n_r: int, r0: float, R: float) -> np.ndarray:
    """r_i = r0 (R / r0)^(i / (n_r - 1)); n_r - 1 must be a multiple of 4."""
    return r0 * (R / r0) ** (np.arange(n_r) / (n_r - 1))


def radial(n_r: int, r0: float, R: float, v, l: int, e: float):
    """Radial function of eq. simp_Schr and its energy derivative (Hartree units) for the spherical
    potential v on the mesh.  Returns (P, Pd) on the even mesh points and the dict of boundary
    values u, du, ud, dud (at R) and ud_norm2."""
    if (n_r - 1) % 4:
        raise ValueError("n_r - 1 must be a multiple of 4")
    v = _c(v, np.float64)
    ne = (n_r - 1) // 2 + 1
    P = np.zeros(ne)
    Pd = np.zeros(ne)
    out = np.zeros(5)
    _load().or_radial(n_r, float(r0), float(R), _p(v), int(l), float(e), _p(P), _p(Pd), _p(out))
    return P, Pd, dict(zip(("u", "du", "ud", "dud", "ud_norm2"), out.tolist()))


def radial_integral(n_r: int, r0: float, R: float, fa, v, fb) -> float:
    """Integral over [r0, R] of fa v fb dr, all on the even mesh points (Simpson's rule in ln r)."""
    fa, v, fb = _c(fa, np.float64), _c(v, np.float64), _c(fb, np.float64)
    return _load().or_radial_integral(n_r, float(r0), float(R), _p(fa), _p(v), _p(fb))


def radial_setup(n_r: int, r0, rmt, v0, e_l, lmax, vlm, lpot: int):
    """Everything the radial data and the potential descriptors need, per type: boundary values,
    ||udot||^2 and the four integral arrays I[type][l'][l][L''] of eq. nonsph_integrals
    (x_{l'} v_{L''} y_l integrated, x, y in {u, udot}).
    v0: (n_types, n_r) spherical potential; vlm: (n_types, (lpot+1)^2, n_r) non-spherical
    components; lmax per type; lstride = max lmax + 1."""
    nt = len(lmax)
    ls = int(max(lmax)) + 1
    nlp = (lpot + 1) ** 2
    out = {k: np.zeros((nt, ls)) for k in ("u", "du", "ud", "dud", "ud_norm2")}
    ints = {k: np.zeros((nt, ls, ls, nlp)) for k in ("i_uu", "i_ud", "i_du", "i_dd")}
    for t in range(nt):
        fun = {}
        for l in range(int(lmax[t]) + 1):
            P, Pd, b = radial(n_r, r0[t], rmt[t], v0[t], l, e_l[t][l])
            fun[l] = (P, Pd)
            for k, val in b.items():
                out[k][t, l] = val
        for L2 in range(nlp):
            ve = np.asarray(vlm[t][L2])[::2]
            for lp in range(int(lmax[t]) + 1):
                for l in range(int(lmax[t]) + 1):
                    (Pp, Pdp), (Pl, Pdl) = fun[lp], fun[l]
                    ints["i_uu"][t, lp, l, L2] = radial_integral(n_r, r0[t], rmt[t], Pp, ve, Pl)
                    ints["i_ud"][t, lp, l, L2] = radial_integral(n_r, r0[t], rmt[t], Pp, ve, Pdl)
                    ints["i_du"][t, lp, l, L2] = radial_integral(n_r, r0[t], rmt[t], Pdp, ve, Pl)
                    ints["i_dd"][t, lp, l, L2] = radial_integral(n_r, r0[t], rmt[t], Pdp, ve, Pdl)
    out.update(ints)
    return out
