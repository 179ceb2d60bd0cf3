"""GPU parity of the modular split precision (residues modulo pairwise coprime moduli <= 255 on
the int8 matrix cores, each complex product split into two real ones, rebuilt by the Chinese remainder theorem) against the FP64 oracle.

Bar: relative Frobenius error <= 1e-10 per matrix (H and S separately) with the default 11
moduli; the error falls with every extra modulus, within 2^(10-B) where B is the integer bit
width the moduli allow."""
import math

import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-10


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_06589_amd import Flapw
    f = Flapw()
    yield f
    f.close()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _mixed(seed=12, n_g=517, n_k=1):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 9.0, size=(5, 3))
    return synthcells.custom_cell("mixed", 9.0, pos, np.array([0, 1, 0, 2, 1], np.int32), [5, 3, 8], [2.0, 1.7, 1.5],
                                  4, [n_g + 37 * i for i in range(n_k)], [seed], rotations="random")


def _upper(M):
    U = np.triu(M.T)
    return U + np.triu(U, 1).conj().T


def _relfro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _rel_err(got, ref):
    """The larger of the relative Frobenius error and the largest entry error relative to the
    largest entry: a bound on either alone would let the other slip."""
    e = float(np.abs(got - ref).max() / np.abs(ref).max()) if np.abs(ref).max() > 0 else float(np.abs(got).max())
    return max(_relfro(got, ref), e)



def _has_sqrt_minus_one(c):
    return any((x * x + 1) % c == 0 for x in range(1, c))


def _bits(nm):
    """Integer width B (rounded down) for nm moduli (pairwise coprime odd numbers <= 255 in which -1
    is a square, taken greedily from 255 down); the columns are scaled to a norm of about 2^B."""
    mods, c = [], 255
    while len(mods) < nm:
        if _has_sqrt_minus_one(c) and all(math.gcd(c, m) == 1 for m in mods):
            mods.append(c)
        c -= 2
    return min(50, int(math.floor((sum(math.log2(m) for m in mods) - 1) / 2)))


def _full_errors(ctx, oracle_lib, cell, slices=0):
    out = ctx.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs], prec="i8mod", slices=slices)
    errs = []
    for ik, (H, S) in enumerate(out):
        Ho, So = oracle_lib.hs_full(cell, ik)
        errs.append((_rel_err(_upper(H.cpu().numpy()), Ho), _rel_err(_upper(S.cpu().numpy()), So)))
    return errs, out


@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_mod_full(ctx, oracle_lib, which):
    print(f"i8mod full {which}", flush=True)
    cell = synthcells.config(0) if which == "c0" else _mixed()
    errs, out = _full_errors(ctx, oracle_lib, cell)
    for eh, es in errs:
        assert eh < TOL_SPLIT and es < TOL_SPLIT, (eh, es)
    H, S = out[0]
    assert np.all(np.diag(H.cpu().numpy()).imag == 0.0)
    assert np.all(np.diag(S.cpu().numpy()).imag == 0.0)


def test_mod_lower_untouched(ctx):
    import torch
    cell = _mixed(n_g=200)
    n = cell.n_g(0)
    sentinel = complex(-2.0, 5.0)
    H = torch.full((n, n + 5), sentinel, dtype=torch.complex128, device="cuda")
    S = torch.full((n, n + 5), sentinel, dtype=torch.complex128, device="cuda")
    ctx.hs_generate(cell, cell.kpts, [_dev(cell.gvecs[0])], prec="i8mod", out=[(H, S)])
    for M in (H.cpu().numpy(), S.cpu().numpy()):
        low = np.tril(np.ones((n, n), bool), -1).T
        assert np.all(M[:, :n][low] == sentinel)
        assert np.all(M[:, n:] == sentinel)


def test_mod_moduli_monotone(ctx, oracle_lib):
    """The error falls with every extra modulus down to the FP64 floor; 11 moduli meet the bar."""
    cell = _mixed(n_g=300)
    prev = None
    for nm in range(8, 15):
        (eh, es), = _full_errors(ctx, oracle_lib, cell, slices=nm)[0]
        e = max(eh, es)
        print(f"moduli {nm}: B {_bits(nm)} err {e:.3e}", flush=True)
        assert e < 2.0 ** (10 - _bits(nm)) + 1e-14, (nm, e)
        if prev is not None and prev > 1e-13:
            assert e < prev / 4, (nm, e, prev)
        if nm == 11:
            assert e < TOL_SPLIT
        prev = e


def test_mod_batched_mixed_lmax(ctx, oracle_lib):
    cell = _mixed(seed=21, n_g=190, n_k=3)
    errs, _ = _full_errors(ctx, oracle_lib, cell)
    for eh, es in errs:
        assert eh < TOL_SPLIT and es < TOL_SPLIT


def test_mod_contract_random_operands(ctx, oracle_lib):
    cell = _mixed(n_g=260)
    A, B = synthcells.random_contraction_inputs([9, 9], cell.k_rows(), 260)
    T = ctx.build_T(cell)
    H, S = ctx.hs_contract(cell, _dev(A.T), _dev(B.T), T, prec="i8mod")
    Ho, So = oracle_lib.hs_block(cell, oracle_lib.tmat_all(cell), A, B, A, B)
    assert _rel_err(_upper(H.cpu().numpy()), Ho) < TOL_SPLIT
    assert _rel_err(_upper(S.cpu().numpy()), So) < TOL_SPLIT


@pytest.mark.parametrize("nm", [8, 14])
def test_mod_single_entry_columns(ctx, oracle_lib, nm):
    """Every column of P = [A; B] has one nonzero entry, so the column scaling turns it into an
    integer within 2^-7 of 2^B: the largest magnitudes the residue step sees (B = 50 at 14 moduli),
    with mantissas up to 2 - 2^-40, signs and phases of all kinds, and magnitudes spread
    over 2^-30..2^30 between columns.  A residue off by one modulus would come back from the
    reconstruction as an error of order M/p relative to the scaled product, far above the bound."""
    print(f"i8mod single-entry columns, {nm} moduli", flush=True)
    cell = _mixed(n_g=200)
    k, n = cell.k_rows(), 200
    rng = np.random.default_rng(31 + nm)
    rows = rng.integers(0, k, size=n)
    mant = rng.uniform(1.0, 2.0, size=n)
    mant[:16] = 2.0 - 2.0 ** -40
    val = mant * 2.0 ** rng.integers(-30, 31, size=n) * np.exp(2j * np.pi * rng.uniform(size=n))
    val[16:24] = mant[16:24] * np.array([1, -1, 1j, -1j, 1, -1, 1j, -1j]) * 2.0 ** 7   # real or imaginary only
    A = np.zeros((k, n), np.complex128)
    B = np.zeros((k, n), np.complex128)
    cols = np.arange(n)
    A[rows[0::2], cols[0::2]] = val[0::2]
    B[rows[1::2], cols[1::2]] = val[1::2]
    T = ctx.build_T(cell)
    H, S = ctx.hs_contract(cell, _dev(A.T), _dev(B.T), T, prec="i8mod", slices=nm)
    Ho, So = oracle_lib.hs_block(cell, oracle_lib.tmat_all(cell), A, B, A, B)
    eh, es = _rel_err(_upper(H.cpu().numpy()), Ho), _rel_err(_upper(S.cpu().numpy()), So)
    print(f"  B {_bits(nm)}: H {eh:.3e} S {es:.3e}", flush=True)
    assert eh < 2.0 ** (8 - _bits(nm)) and es < 2.0 ** (8 - _bits(nm)), (eh, es)


@pytest.mark.parametrize("lnonsph", [-1, 3])
def test_mod_with_legendre_s(ctx, oracle_lib, lnonsph):
    """S by the addition theorem (FP64) and H by the modular contraction, dense and structured T."""
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=31, n_g=333, n_k=2)
    with Flapw() as f:
        f.set_s_method("legendre")
        f.set_lnonsph(lnonsph)
        out = f.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs], prec="i8mod")
        for ik, (H, S) in enumerate(out):
            Ho, So = oracle_lib.hs_full(cell, ik, lnonsph=lnonsph)
            assert _rel_err(_upper(H.cpu().numpy()), Ho) < TOL_SPLIT
            assert _rel_err(_upper(S.cpu().numpy()), So) < 1e-12


def _sampled(ctx, oracle_lib, cell, nsamp=48):
    out = ctx.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs], prec="i8mod")
    T = oracle_lib.tmat_all(cell)
    errs = []
    for ik, (H, S) in enumerate(out):
        n = cell.n_g(ik)
        rng = np.random.default_rng(300 + ik)
        idx = np.unique(np.concatenate([rng.choice(n, nsamp, replace=False), [0, n - 1]]))
        Ho, So = oracle_lib.hs_sampled(cell, ik, idx, idx, T)
        up = idx[:, None] <= idx[None, :]
        for M, R in ((H.cpu().numpy(), Ho), (S.cpu().numpy(), So)):
            got = M[np.ix_(idx, idx)].T
            errs.append(float(np.linalg.norm((got - R)[up]) / np.linalg.norm(R[up])))
    return errs


def test_mod_c1_sampled(ctx, oracle_lib):
    errs = _sampled(ctx, oracle_lib, synthcells.config(1))
    assert max(errs) < TOL_SPLIT, errs


def test_mod_c3_subset_sampled(ctx, oracle_lib):
    errs = _sampled(ctx, oracle_lib, synthcells.config(3, n_k=3), nsamp=32)
    assert max(errs) < TOL_SPLIT, errs


def test_mod_c2_sampled(ctx, oracle_lib):
    """The 256-atom precision workload (l_max 10, l'' 8, N = 6000) on sampled entries."""
    errs = _sampled(ctx, oracle_lib, synthcells.config(2), nsamp=40)
    assert max(errs) < TOL_SPLIT, errs


def test_mod_stage_depths_agree(ctx):
    """The contraction kernel with 32-row LDS stages (four ring buffers) returns the same H and S,
    bit for bit, as with 64-row stages (three buffers): the sums modulo each p are exact either way."""
    import os
    cell = _mixed(seed=19, n_g=421, n_k=2)
    g = [_dev(x) for x in cell.gvecs]
    ref = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec="i8mod")]
    os.environ["FLAPW_MOD_STAGE_ROWS"] = "32"
    try:
        got = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec="i8mod")]
    finally:
        del os.environ["FLAPW_MOD_STAGE_ROWS"]
    for ik, ((a, b), (c, d)) in enumerate(zip(ref, got)):
        up = np.triu(np.ones((cell.n_g(ik), cell.n_g(ik)), bool)).T
        assert np.array_equal(a[up], c[up]) and np.array_equal(b[up], d[up]), ik
