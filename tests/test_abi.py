"""Host-side checks of the C-ABI library (no GPU needed): the library loads, exports every
symbol the header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synthcells

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flapw.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1602_06589_amd import build, flapw
    if not os.path.exists(flapw.LIB_PATH):
        build.build()
    return flapw.load_library()


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(flapw_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_header_symbols_exported(lib):
    from paper_1602_06589_amd import flapw
    declared = _declared()
    assert set(declared) == set(flapw.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", flapw.LIB_PATH], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in declared:
        assert name in syms, name
        assert hasattr(lib, name)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert lib.flapw_status_string(s)
    assert lib.flapw_status_string(-2) == b"vanishing Wronskian"


@pytest.fixture()
def handle(lib):
    from paper_1602_06589_amd.flapw import Flapw
    f = Flapw()
    yield f
    f.close()


class _FakeTensor:
    """Stands in for a device tensor in calls that must fail before any device access."""

    def __init__(self, shape, ptr=0x1000):
        self.shape = shape
        self._p = ptr
        self.device = "cpu"

    def data_ptr(self):
        return self._p


def _call_coeffs(f, cell, ld=None, n_g=None):
    from paper_1602_06589_amd import flapw as F
    f._keep = []
    rad, at = f._radial(cell), f._atoms(cell)
    k = np.zeros(3)
    n = cell.n_g(0) if n_g is None else n_g
    return f._lib.flapw_coeffs(f._h, F._ptr(k), n, ctypes.c_void_p(0x1000), ctypes.byref(at), ctypes.byref(rad),
                               ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                               cell.k_rows() if ld is None else ld, ctypes.c_void_p(0))


def test_validation_ld_and_sizes(handle):
    cell = synthcells.config(0)
    assert _call_coeffs(handle, cell, ld=cell.k_rows() - 1) == -1
    assert b"ld" in handle._lib.flapw_last_error(handle._h)
    assert _call_coeffs(handle, cell, n_g=0) == -1


def test_validation_wronskian(handle):
    cell = synthcells.config(0)
    cell.u[0, 3] = cell.ud[0, 3] * cell.du[0, 3] / cell.dud[0, 3]      # W = 0 exactly
    assert _call_coeffs(handle, cell) == -2


def test_validation_rotation(handle):
    cell = synthcells.config(0)
    cell.rot[1, 0, 0] = 1.01
    assert _call_coeffs(handle, cell) == -1


def test_validation_lmax_cap(handle):
    cell = synthcells.config(0)
    cell.lmax[0] = 13
    assert _call_coeffs(handle, cell) == -1


def test_no_device_after_validation(handle):
    """On a machine without a GPU a valid call reaches the device check and reports it."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cell = synthcells.config(0)
    assert _call_coeffs(handle, cell) == -5


def _call_build_T(f, cell):
    f._keep = []
    rad, pot = f._radial(cell), f._potential(cell)
    ldt = 2 * int((cell.lmax.max() + 1) ** 2)
    return f._lib.flapw_build_T(f._h, ctypes.byref(rad), ctypes.byref(pot), ctypes.c_void_p(0x1000), ldt,
                                ctypes.c_void_p(0))


def test_validation_not_hermitian(handle):
    cell = synthcells.config(0)
    cell.i_uu[0, 2, 3, 5] += 1e-3                                      # breaks (l', l) symmetry
    assert _call_build_T(handle, cell) == -3
    cell = synthcells.config(0)
    cell.i_ud[0, 2, 3, 5] += 1e-3                                      # breaks I^{udot u} = I^{u udot}^T
    assert _call_build_T(handle, cell) == -3
    cell = synthcells.config(0)
    cell.i_dd[0, 2, 2, 5] += 1e-3                                      # breaks the reality rule in m''
    assert _call_build_T(handle, cell) == -3


def test_validation_lpot(handle):
    cell = synthcells.config(0)
    cell.lpot = 13
    assert _call_build_T(handle, cell) == -1


def _gen_args(f, cell, n_g=None):
    """Argument tuple of flapw_hs_generate / flapw_plan_create up to (but excluding) prec, with
    stand-in device pointers (the calls must fail before touching them)."""
    from paper_1602_06589_amd import flapw as F
    f._keep = []
    n = np.array([cell.n_g(0) if n_g is None else n_g], np.int32)
    k = np.zeros(3)
    ptrs = [(ctypes.c_void_p * 1)(0x1000 * (i + 1)) for i in range(3)]
    ld = np.array([max(int(n[0]), 1)], np.int64)
    rad, at, pot = f._radial(cell), f._atoms(cell), f._potential(cell)
    f._keep += [n, k, ptrs, ld, rad, at, pot]
    return (f._h, 1, F._ptr(k), F._ptr(n), ptrs[0], ctypes.byref(at), ctypes.byref(rad), ctypes.byref(pot), ptrs[1],
            ptrs[2], F._ptr(ld))


def test_plan_validation(handle):
    cell = synthcells.config(0)
    out = ctypes.c_void_p(0x1234)
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell, n_g=0), 0, 0, ctypes.byref(out)) == -1
    assert out.value is None                                          # cleared on failure
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 1, 2, ctypes.byref(out)) == -6
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 3, 7, ctypes.byref(out)) == -6
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 5, 0, ctypes.byref(out)) == -1
    # modular split: 8..14 moduli; 1..7 unsupported, beyond the cap an argument error
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 4, 7, ctypes.byref(out)) == -6
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 4, 15, ctypes.byref(out)) == -1
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 4, -1, ctypes.byref(out)) == -1
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 0, 0, None) == -1
    assert handle._lib.flapw_plan_launch(None, None) == -1
    assert handle._lib.flapw_plan_destroy(None) == -1


def test_precision_enum(handle, lib):
    """flapw_prec as the boundary names it: 0 FP64, 1 SPLIT_BF16, 2 SPLIT_FP32 (reserved: every call
    returns FLAPW_ERR_UNSUPPORTED), 3 SPLIT_I8, 4 SPLIT_I8_MOD; anything else is an argument error.
    Valid precisions pass validation (without a device they stop at the device check)."""
    import torch
    from paper_1602_06589_amd import flapw as F
    assert (F.FP64, F.SPLIT_BF16, F.SPLIT_FP32, F.SPLIT_I8, F.SPLIT_I8_MOD) == (0, 1, 2, 3, 4)
    cell = synthcells.config(0)
    gen = lambda prec, sl=0: lib.flapw_hs_generate(*_gen_args(handle, cell), prec, sl, None)
    assert gen(2) == -6 and gen(2, 2) == -6
    assert b"FP32" in lib.flapw_last_error(handle._h)
    out = ctypes.c_void_p()
    assert lib.flapw_plan_create(*_gen_args(handle, cell), 2, 0, ctypes.byref(out)) == -6
    assert _call_tune(handle, cell, 1e-10, prec=2)[0] == -6
    for bad in (-1, 5, 99):
        assert gen(bad) == -1
    if not torch.cuda.is_available():
        for good in (0, 1, 3, 4):
            assert gen(good) == -5
    # counts: digits 3..6 for 1 and 3, moduli 8..14 for 4
    assert gen(1, 7) == -6 and gen(3, 2) == -6 and gen(4, 7) == -6 and gen(4, 15) == -1
    # flapw_hs_contract rejects the reserved precision before touching its (stand-in) pointers
    handle._keep = []
    rad, at = handle._radial(cell), handle._atoms(cell)
    P = ctypes.c_void_p
    n, kr = cell.n_g(0), cell.k_rows()
    assert lib.flapw_hs_contract(handle._h, n, ctypes.byref(at), ctypes.byref(rad), P(0x1000), P(0x2000), kr,
                                 P(0x3000), 2 * 49, P(0x4000), P(0x5000), n, 2, 0, None) == -6


def _call_tune(f, cell, tol, prec=3, n_g=None):
    from paper_1602_06589_amd import flapw as F
    f._keep = []
    rad, at, pot = f._radial(cell), f._atoms(cell), f._potential(cell)
    k = np.zeros(3)
    sl, band = ctypes.c_int(-1), ctypes.c_int(-1)
    err = (ctypes.c_double * 4)()
    st = f._lib.flapw_tune(f._h, F._ptr(k), cell.n_g(0) if n_g is None else n_g, ctypes.c_void_p(0x1000),
                           ctypes.byref(at), ctypes.byref(rad), ctypes.byref(pot), prec, tol, ctypes.byref(sl),
                           ctypes.byref(band), None, err, None)
    return st, sl.value, band.value


def test_tune_validation(handle):
    cell = synthcells.config(0)
    assert _call_tune(handle, cell, 0.0)[0] == -1
    assert _call_tune(handle, cell, float("nan"))[0] == -1
    assert _call_tune(handle, cell, 1e-10, n_g=0)[0] == -1
    assert _call_tune(handle, cell, 1e-10, prec=5)[0] == -1
    assert _call_tune(handle, cell, 1e-10, prec=2)[0] == -6           # FP32 slices: reserved
    bad = synthcells.config(0)
    bad.i_uu[0, 2, 3, 5] += 1e-3
    assert _call_tune(handle, bad, 1e-10)[0] == -3


def test_plan_and_tune_no_device(handle):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cell = synthcells.config(0)
    out = ctypes.c_void_p()
    assert handle._lib.flapw_plan_create(*_gen_args(handle, cell), 3, 0, ctypes.byref(out)) == -5
    st, sl, band = _call_tune(handle, cell, 1e-10)
    assert st == -5 and sl == -1 and band == -1                       # outputs untouched on failure


def test_handle_settings_validation(handle):
    lib = handle._lib
    assert lib.flapw_set_lnonsph(handle._h, -2) == -1
    assert lib.flapw_set_lnonsph(handle._h, 13) == -1
    assert lib.flapw_set_lnonsph(handle._h, -1) == 0
    assert lib.flapw_set_lnonsph(handle._h, 12) == 0
    assert lib.flapw_set_s_method(handle._h, 2) == -1
    assert lib.flapw_set_s_method(handle._h, 1) == 0
    assert lib.flapw_set_s_method(None, 0) == -1
    assert lib.flapw_set_lnonsph(None, 0) == -1


def test_s_legendre_validation(handle):
    from paper_1602_06589_amd import flapw as F
    cell = synthcells.config(0)
    handle._keep = []
    rad, at = handle._radial(cell), handle._atoms(cell)
    k = np.zeros(3)
    call = lambda n, lds, S=0x2000: handle._lib.flapw_s_legendre(handle._h, F._ptr(k), n, ctypes.c_void_p(0x1000),
                                                                 ctypes.byref(at), ctypes.byref(rad),
                                                                 ctypes.c_void_p(S), lds, None)
    assert call(0, 10) == -1
    assert call(10, 9) == -1
    assert call(10, 10, S=0) == -1
    cell.u[0, 1] = cell.ud[0, 1] * cell.du[0, 1] / cell.dud[0, 1]       # W = 0
    handle._keep = []
    rad = handle._radial(cell)
    assert call(10, 10) == -2


def _mesh_args(handle, m, **over):
    from paper_1602_06589_amd import flapw as F
    f = dict(n_types=len(m.lmax), lstride=m.e_l.shape[1], lmax=m.lmax, rmt=m.rmt, r0=m.r0, n_r=m.n_r, e_l=m.e_l,
             v_sph=m.v_sph, lpot=m.lpot, v_lm=m.v_lm)
    f.update(over)
    arrs = {k: (F._i32(v) if k == "lmax" else F._f64(v)) for k, v in f.items() if isinstance(v, np.ndarray)}
    handle._keep = list(arrs.values())
    mesh = F._RadialMesh(f["n_types"], f["lstride"], F._ptr(arrs["lmax"]), F._ptr(arrs["rmt"]), F._ptr(arrs["r0"]),
                         f["n_r"], F._ptr(arrs["e_l"]), F._ptr(arrs["v_sph"]), f["lpot"], F._ptr(arrs["v_lm"]))
    handle._keep.append(mesh)
    nt, ls, nlp = f["n_types"], f["lstride"], (max(f["lpot"], 0) + 1) ** 2
    outs = [np.full((max(nt, 1), ls), 7.0) for _ in range(5)] + [np.full((max(nt, 1), ls, ls, nlp), 7.0) for _ in range(4)]
    handle._keep += outs
    return mesh, outs


def test_radial_setup_validation(handle):
    from paper_1602_06589_amd import flapw as F
    m = synthcells.radial_meshes([3, 2], [2.0, 2.3], 2, n_r=41, seed=1)
    lib = handle._lib

    def call(**over):
        mesh, outs = _mesh_args(handle, m, **over)
        st = lib.flapw_radial_setup(handle._h, ctypes.byref(mesh), *[F._ptr(o) for o in outs], None)
        assert all(np.all(o == 7.0) for o in outs)          # nothing written on error
        return st

    assert lib.flapw_radial_setup(handle._h, None, *([None] * 9), None) == -1
    assert call(n_r=43) == -1                               # n_r - 1 not a multiple of 4
    assert call(n_r=5, v_sph=m.v_sph[:, :5], v_lm=m.v_lm[:, :, :5]) == -1
    assert call(lstride=3) == -1                            # < max lmax + 1
    assert call(lpot=13) == -1
    assert call(lmax=np.array([13, 2])) == -1
    assert call(r0=np.array([2.5, 1e-6])) == -1              # r0 >= R
    assert call(r0=np.array([1e-11, 1e-6])) == -1
    bad = m.v_sph.copy()
    bad[1, 7] = np.nan
    assert call(v_sph=bad) == -1
    bad = m.e_l.copy()
    bad[0, 3] = np.inf
    assert call(e_l=bad) == -1
    bad = m.v_lm.copy()
    bad[0, 1, 10] += 1e-3                                   # v(1,-1) != -v(1,1)
    assert call(v_lm=bad) == -3
    # valid arguments: without a device the call fails with FLAPW_ERR_DEVICE, else succeeds
    st = call() if not _has_device() else None
    if st is not None:
        assert st == -5


def _has_device():
    import torch
    return torch.cuda.device_count() > 0


def test_release_workspace(handle, lib):
    """Releasing the work buffers of a handle leaves it usable and holding nothing; a NULL handle
    is an argument error."""
    handle.release_workspace()
    assert handle.workspace_bytes == 0
    handle.release_workspace()
    assert lib.flapw_release_workspace(None) == -1
    assert lib.flapw_set_workspace_limit(None, 0) == -1
    assert lib.flapw_set_workspace_limit(handle._h, 1 << 30) == 0
    assert lib.flapw_set_workspace_limit(handle._h, -5) == 0


def test_interstitial_validation(handle, lib):
    """flapw_interstitial and flapw_set_interstitial reject overlapping spheres, a lattice that does
    not hold omega, NULL pointers and bad sizes before touching the device."""
    from paper_1602_06589_amd import flapw as F
    import torch
    P = ctypes.c_void_p
    k = np.zeros(3)

    def call(cell, lat=None, n=None, ldh=None, v=0.0):
        handle._keep = []
        rad, at = handle._radial(cell), handle._atoms(cell)
        la = F._f64(cell.lattice if lat is None else lat)
        handle._keep += [la]
        nn = cell.n_g(0) if n is None else n
        return lib.flapw_interstitial(handle._h, F._ptr(k), nn, P(0x1000), ctypes.byref(at), ctypes.byref(rad),
                                      F._ptr(la), v, P(0x2000), P(0x3000), nn if ldh is None else ldh, None)

    over = synthcells.config(0)                                      # two spheres 0.8 bohr apart
    assert synthcells.min_sphere_gap(over) < 0
    assert call(over) == -1
    assert b"overlap" in lib.flapw_last_error(handle._h)
    sep = synthcells.config_separated(0)
    assert call(sep, lat=sep.lattice * 1.01) == -1                   # |det| != omega
    assert call(sep, n=0) == -1
    assert call(sep, ldh=10) == -1
    assert call(sep, v=float("nan")) == -1
    # a sphere overlapping its own periodic image
    big = synthcells.custom_cell("img", 3.0, np.array([[1.0, 1.0, 1.0]]), np.zeros(1, np.int32), [2], [1.6], 2, 20,
                                 [3])
    assert call(big) == -1
    if not torch.cuda.is_available():
        assert call(sep) == -5
    assert lib.flapw_set_interstitial(handle._h, 1, None, 0.0) == -1
    assert lib.flapw_set_interstitial(handle._h, 0, None, float("inf")) == -1
    la = F._f64(over.lattice)
    assert lib.flapw_set_interstitial(handle._h, 1, F._ptr(la), 0.0) == 0
    # with the setting on, generation validates the spheres too
    assert lib.flapw_hs_generate(*_gen_args(handle, over), 0, 0, None) == -1
    assert b"overlap" in lib.flapw_last_error(handle._h)
    assert lib.flapw_set_interstitial(handle._h, 0, None, 0.0) == 0


def test_eigensolve_validation(handle, lib):
    import torch
    P = ctypes.c_void_p
    assert lib.flapw_eigensolve(handle._h, 0, P(0x1000), 1, P(0x2000), 1, P(0x3000), 1, None) == -1
    assert lib.flapw_eigensolve(handle._h, 10, P(0x1000), 9, P(0x2000), 10, P(0x3000), 1, None) == -1
    assert lib.flapw_eigensolve(handle._h, 10, None, 10, P(0x2000), 10, P(0x3000), 1, None) == -1
    assert lib.flapw_eigensolve(handle._h, 10, P(0x1000), 10, P(0x2000), 10, None, 1, None) == -1
    if not torch.cuda.is_available():
        assert lib.flapw_eigensolve(handle._h, 10, P(0x1000), 10, P(0x2000), 10, P(0x3000), 1, None) == -5
    for s in (-7, -8):
        assert lib.flapw_status_string(s) != b"unknown status"
