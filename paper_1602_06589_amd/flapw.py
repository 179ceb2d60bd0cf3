"""Python binding of the C-ABI in include/flapw.h (argument marshalling only).

Every computation runs in the HIP library ``libflapw_hip.so`` built next to this file; torch
supplies device memory (complex128 tensors) and the current HIP stream.  There is no
fallback: if the library is missing or the GPU is absent the calls raise.

Array conventions (all dense matrices are column-major, as the library's):
  A, B   torch complex128 tensors of shape (n_g, ld): row t is column t of the K x n_g matrix
  T      torch complex128 tensor of shape (n_types, ldt, ldt): T[tau][c][r] is entry (r, c)
  H, S   torch complex128 tensors of shape (n_g, ldh): H[t][r] is entry (r, t); only r <= t is
         written.  ``hermitian_full`` expands such a tensor to the full matrix.

A `system` argument is any object with the attributes of a FLAPW problem:
  lmax (n_types,) int, rmt, u, du, ud, dud, ud_norm2, e_l ((n_types, lstride) float),
  atom_type (n_atoms,) int, pos (n_atoms, 3), rot (n_atoms, 3, 3), omega,
  lpot and i_uu, i_ud, i_du, i_dd ((n_types, lstride, lstride, (lpot+1)^2) float).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflapw_hip.so")

FP64, SPLIT_BF16, SPLIT_FP32, SPLIT_I8, SPLIT_I8_MOD = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "bf16": SPLIT_BF16, "fp32": SPLIT_FP32, "i8": SPLIT_I8, "i8mod": SPLIT_I8_MOD}
S_METHODS = {"gemm": 0, "legendre": 1}

_STATUS = {0: "FLAPW_OK", -1: "FLAPW_ERR_ARG", -2: "FLAPW_ERR_WRONSKIAN", -3: "FLAPW_ERR_NOT_HERMITIAN",
           -4: "FLAPW_ERR_NOMEM", -5: "FLAPW_ERR_DEVICE", -6: "FLAPW_ERR_UNSUPPORTED", -7: "FLAPW_ERR_NOT_POSDEF",
           -8: "FLAPW_ERR_NO_CONVERGENCE"}

EXPORTS = ["flapw_create", "flapw_destroy", "flapw_status_string", "flapw_last_error", "flapw_workspace_bytes",
           "flapw_release_workspace",
           "flapw_coeffs", "flapw_build_T", "flapw_hs_contract", "flapw_hs_generate", "flapw_set_s_method",
           "flapw_set_lnonsph", "flapw_s_legendre", "flapw_plan_create",
           "flapw_plan_launch", "flapw_plan_destroy", "flapw_tune", "flapw_profile_enable", "flapw_profile_query",
           "flapw_radial_setup", "flapw_hs_contract_noalloc", "flapw_noalloc_scratch_bytes", "flapw_interstitial",
           "flapw_set_interstitial", "flapw_eigensolve", "flapw_set_workspace_limit"]


class FlapwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class _Radial(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int), ("lstride", ctypes.c_int), ("lmax", ctypes.c_void_p),
                ("rmt", ctypes.c_void_p), ("u", ctypes.c_void_p), ("du", ctypes.c_void_p), ("ud", ctypes.c_void_p),
                ("dud", ctypes.c_void_p), ("ud_norm2", ctypes.c_void_p), ("e_l", ctypes.c_void_p)]


class _RadialMesh(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int), ("lstride", ctypes.c_int), ("lmax", ctypes.c_void_p),
                ("rmt", ctypes.c_void_p), ("r0", ctypes.c_void_p), ("n_r", ctypes.c_int), ("e_l", ctypes.c_void_p),
                ("v_sph", ctypes.c_void_p), ("lpot", ctypes.c_int), ("v_lm", ctypes.c_void_p)]


class _Atoms(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int), ("type", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("rot", ctypes.c_void_p), ("omega", ctypes.c_double)]


class _Potential(ctypes.Structure):
    _fields_ = [("lpot", ctypes.c_int), ("i_uu", ctypes.c_void_p), ("i_ud", ctypes.c_void_p),
                ("i_du", ctypes.c_void_p), ("i_dd", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libflapw_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is missing: build it with paper_1602_06589_amd/build.py")
        # torch first: its HIP runtime must be the one the library binds to (one runtime per process)
        import torch  # noqa: F401
        lib = ctypes.CDLL(path)
        P, I, L = ctypes.c_void_p, ctypes.c_int, ctypes.c_long
        lib.flapw_create.argtypes = [ctypes.POINTER(P)]
        lib.flapw_destroy.argtypes = [P]
        lib.flapw_status_string.argtypes = [I]
        lib.flapw_status_string.restype = ctypes.c_char_p
        lib.flapw_last_error.argtypes = [P]
        lib.flapw_last_error.restype = ctypes.c_char_p
        lib.flapw_workspace_bytes.argtypes = [P]
        lib.flapw_workspace_bytes.restype = ctypes.c_longlong
        lib.flapw_release_workspace.argtypes = [P]
        lib.flapw_set_workspace_limit.argtypes = [P, ctypes.c_longlong]
        lib.flapw_release_workspace.restype = ctypes.c_int
        lib.flapw_coeffs.argtypes = [P, P, I, P, P, P, P, P, L, P]
        lib.flapw_build_T.argtypes = [P, P, P, P, L, P]
        lib.flapw_hs_contract.argtypes = [P, I, P, P, P, P, L, P, L, P, P, L, I, I, P]
        lib.flapw_hs_contract_noalloc.argtypes = [P, I, P, P, P, P, L, P, L, P, P, L, I, I, P]
        lib.flapw_noalloc_scratch_bytes.argtypes = []
        lib.flapw_noalloc_scratch_bytes.restype = ctypes.c_longlong
        lib.flapw_hs_generate.argtypes = [P, I, P, P, P, P, P, P, P, P, P, I, I, P]
        lib.flapw_set_s_method.argtypes = [P, I]
        lib.flapw_set_lnonsph.argtypes = [P, I]
        lib.flapw_s_legendre.argtypes = [P, P, I, P, P, P, P, L, P]
        lib.flapw_plan_create.argtypes = [P, I, P, P, P, P, P, P, P, P, P, I, I, ctypes.POINTER(P)]
        lib.flapw_plan_launch.argtypes = [P, P]
        lib.flapw_plan_destroy.argtypes = [P]
        D = ctypes.POINTER(ctypes.c_double)
        lib.flapw_tune.argtypes = [P, P, I, P, P, P, P, I, ctypes.c_double, ctypes.POINTER(I), ctypes.POINTER(I),
                                   ctypes.POINTER(I), D, D]
        lib.flapw_profile_enable.argtypes = [P, I]
        lib.flapw_profile_query.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_double)]
        lib.flapw_radial_setup.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
        lib.flapw_interstitial.argtypes = [P, P, I, P, P, P, P, ctypes.c_double, P, P, L, P]
        lib.flapw_set_interstitial.argtypes = [P, I, P, ctypes.c_double]
        lib.flapw_eigensolve.argtypes = [P, I, P, L, P, L, P, I, P]
        for f in EXPORTS:
            getattr(lib, f).restype = getattr(lib, f).restype or ctypes.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream) -> ctypes.c_void_p:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(int(s.cuda_stream))


def _dptr(t) -> int:
    return int(t.data_ptr())


def k_rows(system) -> int:
    lm = np.asarray(system.lmax)[np.asarray(system.atom_type)]
    return int(((lm + 1) ** 2).sum())


def hermitian_full(M):
    """Expand an upper-triangle column-major result tensor (n, ld) to the full (n x n) matrix."""
    import torch
    n = M.shape[0]
    U = torch.triu(M[:, :n].transpose(0, 1))
    return U + torch.triu(U, 1).conj().transpose(0, 1)


class Flapw:
    """One library handle (owns the device work buffers).  Use as a context manager."""

    def __init__(self):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        self._check(self._lib.flapw_create(ctypes.byref(self._h)))
        self._keep = []

    def close(self):
        if self._h:
            self._lib.flapw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            msg = self._lib.flapw_last_error(self._h).decode() if self._h else ""
            raise FlapwError(st, msg)

    def profile(self, on: bool = True):
        """Start (or stop) recording HIP events around every kernel launch; resets the record."""
        self._check(self._lib.flapw_profile_enable(self._h, int(bool(on))))

    def kernel_time(self, family: str):
        """(launches, total milliseconds) of a kernel family since profile(True)."""
        n = ctypes.c_int()
        ms = ctypes.c_double()
        self._check(self._lib.flapw_profile_query(self._h, family.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.flapw_workspace_bytes(self._h))

    def release_workspace(self):
        """Free the handle's work buffers (the next call allocates what it needs again)."""
        self._check(self._lib.flapw_release_workspace(self._h))

    def set_workspace_limit(self, nbytes: int = -1):
        """After a call that leaves the work buffers above nbytes, wait and free them (-1: keep)."""
        self._check(self._lib.flapw_set_workspace_limit(self._h, int(nbytes)))

    # --------------------------------------------------------------------- descriptors
    def _radial(self, s):
        arrs = [_i32(s.lmax), _f64(s.rmt), _f64(s.u), _f64(s.du), _f64(s.ud), _f64(s.dud), _f64(s.ud_norm2),
                _f64(s.e_l)]
        self._keep += arrs
        return _Radial(len(arrs[0]), int(np.asarray(s.u).shape[1]), *[_ptr(a) for a in arrs])

    def _atoms(self, s):
        arrs = [_i32(s.atom_type), _f64(s.pos), _f64(s.rot)]
        self._keep += arrs
        return _Atoms(len(arrs[0]), _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), float(s.omega))

    def _potential(self, s):
        arrs = [_f64(s.i_uu), _f64(s.i_ud), _f64(s.i_du), _f64(s.i_dd)]
        self._keep += arrs
        return _Potential(int(s.lpot), *[_ptr(a) for a in arrs])

    # --------------------------------------------------------------------- calls
    def coeffs(self, system, k, g, A=None, B=None, stream=None):
        """A_*, B_* of one k-point.  g: device tensor (n_g, 3) float64 of Cartesian G."""
        import torch
        self._keep = []
        n_g = int(g.shape[0])
        kr = k_rows(system)
        if A is None:
            A = torch.zeros((n_g, kr), dtype=torch.complex128, device=g.device)
        if B is None:
            B = torch.zeros((n_g, kr), dtype=torch.complex128, device=g.device)
        kk = _f64(k)
        rad, at = self._radial(system), self._atoms(system)
        self._check(self._lib.flapw_coeffs(self._h, _ptr(kk), n_g, _dptr(g), ctypes.byref(at), ctypes.byref(rad),
                                           _dptr(A), _dptr(B), int(A.shape[1]), _stream(stream)))
        return A, B

    def build_T(self, system, ldt: Optional[int] = None, device="cuda", stream=None):
        import torch
        self._keep = []
        nlmax = int((np.max(system.lmax) + 1) ** 2)
        ldt = ldt or 2 * nlmax
        T = torch.empty((len(system.lmax), ldt, ldt), dtype=torch.complex128, device=device)
        rad, pot = self._radial(system), self._potential(system)
        self._check(self._lib.flapw_build_T(self._h, ctypes.byref(rad), ctypes.byref(pot), _dptr(T), ldt,
                                            _stream(stream)))
        return T

    def hs_contract(self, system, A, B, T, prec="fp64", slices: int = 0, H=None, S=None, stream=None,
                    no_alloc: bool = False):
        """S and H from given A, B (tensors (n_g, ld)) and T.  no_alloc: flapw_hs_contract_noalloc (work
        buffers in the library's static per-device scratch; the outputs, when not given, are still
        allocated here by torch)."""
        import torch
        self._keep = []
        n_g = int(A.shape[0])
        if H is None:
            H = torch.zeros((n_g, n_g), dtype=torch.complex128, device=A.device)
        if S is None:
            S = torch.zeros((n_g, n_g), dtype=torch.complex128, device=A.device)
        rad, at = self._radial(system), self._atoms(system)
        fn = self._lib.flapw_hs_contract_noalloc if no_alloc else self._lib.flapw_hs_contract
        self._check(fn(self._h, n_g, ctypes.byref(at), ctypes.byref(rad), _dptr(A), _dptr(B),
                                                int(A.shape[1]), _dptr(T), int(T.shape[-1]), _dptr(H), _dptr(S),
                                                int(H.shape[1]), PRECISIONS.get(prec, prec), int(slices),
                                                _stream(stream)))
        return H, S

    def set_s_method(self, method: str = "gemm"):
        """How hs_generate and plan compute S: "gemm" (with H on the matrix cores, in the chosen
        precision) or "legendre" (addition theorem, FP64; the contraction then computes H only)."""
        self._check(self._lib.flapw_set_s_method(self._h, S_METHODS.get(method, method)))

    def set_lnonsph(self, lnonsph: int = -1):
        """Structured T: non-spherical terms only for l', l <= lnonsph (-1: dense T)."""
        self._check(self._lib.flapw_set_lnonsph(self._h, int(lnonsph)))

    def interstitial(self, system, k, g, H, S, v_int: float = 0.0, stream=None):
        """Adds the interstitial S and H of one k-point to the upper triangles of H and S (tensors
        (n_g, ld)); g: device tensor (n_g, 3).  system needs `lattice` (3 x 3 rows)."""
        self._keep = []
        kk, lat = _f64(k), _f64(system.lattice)
        rad, at = self._radial(system), self._atoms(system)
        self._keep += [kk, lat]
        self._check(self._lib.flapw_interstitial(self._h, _ptr(kk), int(g.shape[0]), _dptr(g), ctypes.byref(at),
                                                 ctypes.byref(rad), _ptr(lat), float(v_int), _dptr(H), _dptr(S),
                                                 int(H.shape[1]), _stream(stream)))
        return H, S

    def set_interstitial(self, on: bool = True, lattice=None, v_int: float = 0.0):
        """Generation (hs_generate, plan) adds the interstitial terms, giving the full H and S."""
        lat = _f64(lattice) if lattice is not None else None
        self._check(self._lib.flapw_set_interstitial(self._h, int(bool(on)), None if lat is None else _ptr(lat),
                                                     float(v_int)))

    def eigensolve(self, H, S, vectors: bool = True, w=None, stream=None):
        """H c = eps S c in place (rocSOLVER zhegvd on the upper triangles): returns (w, H) with the
        eigenvalues ascending and, with vectors, the S-orthonormal eigenvectors in the columns of the
        column-major H (tensor row t = column t); S then holds its Cholesky factor."""
        import torch
        n = int(H.shape[0])
        if w is None:
            w = torch.empty(n, dtype=torch.float64, device=H.device)
        self._check(self._lib.flapw_eigensolve(self._h, n, _dptr(H), int(H.shape[1]), _dptr(S), int(S.shape[1]),
                                               _dptr(w), int(bool(vectors)), _stream(stream)))
        return w, H

    def radial_setup(self, n_r: int, r0, rmt, v_sph, e_l, lmax, v_lm, lpot: int, stream=None):
        """Radial boundary data and the four non-spherical integral tables from radial meshes
        (flapw_radial_setup).  r0, rmt: per type; v_sph: (n_types, n_r); e_l: (n_types, lstride);
        v_lm: (n_types, (lpot+1)^2, n_r).  Returns a dict with u, du, ud, dud, ud_norm2
        (n_types, lstride) and i_uu, i_ud, i_du, i_dd (n_types, lstride, lstride, (lpot+1)^2)."""
        self._keep = []
        lm, r0a, rmta, el = _i32(lmax), _f64(r0), _f64(rmt), _f64(e_l)
        vs, vl = _f64(v_sph), _f64(v_lm)
        nt, ls = int(lm.shape[0]), int(el.shape[1])
        nlp = (int(lpot) + 1) ** 2
        if el.shape != (nt, ls) or vs.shape != (nt, n_r) or vl.shape != (nt, nlp, n_r) or r0a.shape != (nt,) \
                or rmta.shape != (nt,):
            raise ValueError("radial_setup: array shapes do not match n_types, n_r, lpot")
        mesh = _RadialMesh(nt, ls, _ptr(lm), _ptr(rmta), _ptr(r0a), int(n_r), _ptr(el), _ptr(vs), int(lpot), _ptr(vl))
        out = {k: np.zeros((nt, ls)) for k in ("u", "du", "ud", "dud", "ud_norm2")}
        out.update({k: np.zeros((nt, ls, ls, nlp)) for k in ("i_uu", "i_ud", "i_du", "i_dd")})
        self._keep += [lm, r0a, rmta, el, vs, vl, mesh]
        self._check(self._lib.flapw_radial_setup(
            self._h, ctypes.byref(mesh), *[_ptr(out[k]) for k in ("u", "du", "ud", "dud", "ud_norm2", "i_uu", "i_ud",
                                                                   "i_du", "i_dd")], _stream(stream)))
        return out

    def s_legendre(self, system, k, g, S=None, stream=None):
        """S of one k-point through the addition theorem.  g: device tensor (n_g, 3)."""
        import torch
        self._keep = []
        n_g = int(g.shape[0])
        if S is None:
            S = torch.zeros((n_g, n_g), dtype=torch.complex128, device=g.device)
        kk = _f64(k)
        rad, at = self._radial(system), self._atoms(system)
        self._check(self._lib.flapw_s_legendre(self._h, _ptr(kk), n_g, _dptr(g), ctypes.byref(at), ctypes.byref(rad),
                                               _dptr(S), int(S.shape[1]), _stream(stream)))
        return S

    def _generate_args(self, system, kpts, gvecs, out):
        import torch
        self._keep = []
        nk = len(gvecs)
        ng = np.array([int(g.shape[0]) for g in gvecs], dtype=np.int32)
        if out is None:
            out = [(torch.zeros((int(n), int(n)), dtype=torch.complex128, device=gvecs[0].device),
                    torch.zeros((int(n), int(n)), dtype=torch.complex128, device=gvecs[0].device)) for n in ng]
        kk = _f64(np.asarray(kpts).reshape(nk, 3))
        gp = (ctypes.c_void_p * nk)(*[_dptr(g) for g in gvecs])
        hp = (ctypes.c_void_p * nk)(*[_dptr(h) for h, _ in out])
        sp = (ctypes.c_void_p * nk)(*[_dptr(s) for _, s in out])
        ld = np.array([int(h.shape[1]) for h, _ in out], dtype=np.int64)
        rad, at, pot = self._radial(system), self._atoms(system), self._potential(system)
        self._keep += [kk, ng, gp, hp, sp, ld, rad, at, pot]
        return out, (nk, _ptr(kk), _ptr(ng), gp, ctypes.byref(at), ctypes.byref(rad), ctypes.byref(pot), hp, sp,
                     _ptr(ld))

    def hs_generate(self, system, kpts, gvecs: Sequence, prec="fp64", slices: int = 0, out: Optional[List] = None,
                    stream=None):
        """H and S of every k-point.  gvecs: device tensors (n_g_i, 3).  Returns [(H_i, S_i)]."""
        out, args = self._generate_args(system, kpts, gvecs, out)
        self._check(self._lib.flapw_hs_generate(self._h, *args, PRECISIONS.get(prec, prec), int(slices),
                                                _stream(stream)))
        return out

    def plan(self, system, kpts, gvecs: Sequence, prec="fp64", slices: int = 0, out: Optional[List] = None):
        """Captures the generation of hs_generate into a HIP graph; returns a Plan whose launch()
        replays it into the same outputs (Plan.out)."""
        out, args = self._generate_args(system, kpts, gvecs, out)
        handle = ctypes.c_void_p()
        self._check(self._lib.flapw_plan_create(self._h, *args, PRECISIONS.get(prec, prec), int(slices),
                                                ctypes.byref(handle)))
        return Plan(self, handle, out, list(gvecs))

    def tune(self, system, k, g, prec="i8", tol: float = 1e-10):
        """Runs the autotuner on one k-point (g: device tensor (n_g, 3)); the handle keeps the choice.
        Returns {"slices", "band", "stage_rows" (modular path: 64 or 32, else 0), "digit_err"
        (estimated whole-matrix errors for 3..6 digits, or 10..13 moduli for "i8mod"), "band_ms"
        (bands 1, 2, 4, 8, 16 with 64-row stages, then with 32-row stages for "i8mod")}."""
        self._keep = []
        kk = _f64(k)
        rad, at, pot = self._radial(system), self._atoms(system), self._potential(system)
        sl, band, rows = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        err = (ctypes.c_double * 4)()
        ms = (ctypes.c_double * 10)()
        st = self._lib.flapw_tune(self._h, _ptr(kk), int(g.shape[0]), _dptr(g), ctypes.byref(at), ctypes.byref(rad),
                                  ctypes.byref(pot), PRECISIONS.get(prec, prec), float(tol), ctypes.byref(sl),
                                  ctypes.byref(band), ctypes.byref(rows), err, ms)
        res = {"slices": sl.value, "band": band.value, "stage_rows": rows.value, "digit_err": list(err),
               "band_ms": list(ms)}
        if st != 0:
            e = FlapwError(st, self._lib.flapw_last_error(self._h).decode())
            e.result = res
            raise e
        return res


class Plan:
    """A captured H/S generation (see Flapw.plan).  Keeps its outputs and G lists alive."""

    def __init__(self, owner: "Flapw", handle, out, gvecs):
        self._owner, self._p, self.out, self._g = owner, handle, out, gvecs

    def launch(self, stream=None):
        if not self._p:
            raise FlapwError(-1, "plan destroyed")
        self._owner._check(self._owner._lib.flapw_plan_launch(self._p, _stream(stream)))
        return self.out

    def close(self):
        if self._p:
            self._owner._lib.flapw_plan_destroy(self._p)
            self._p = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
