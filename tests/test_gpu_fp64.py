"""GPU parity of the FP64 path against the oracle (called through the C-ABI binding).

Bar (FP64 path): relative Frobenius error <= 1e-12 per matrix (H and S separately) on the
compared entries; coefficients and T elementwise to 1e-13 of their largest magnitude."""
import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


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


def _relfro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _rel_err(got, ref):
    """The larger of the relative Frobenius error and the largest entry error relative to the
    largest entry: a bound on either alone would let the other slip."""
    e = float(np.abs(got - ref).max() / np.abs(ref).max()) if np.abs(ref).max() > 0 else float(np.abs(got).max())
    return max(_relfro(got, ref), e)



def _upper(M):
    """Full Hermitian matrix from an upper-triangle result (entry (r, t) at M[t, r])."""
    U = np.triu(M.T)
    return U + np.triu(U, 1).conj().T


@pytest.mark.parametrize("which", ["c0", "mixed", "c1"])
def test_coeffs_parity(ctx, oracle_lib, which):
    cell = {"c0": lambda: synthcells.config(0), "mixed": _mixed, "c1": lambda: synthcells.config(1)}[which]()
    ik = 0
    A, B = ctx.coeffs(cell, cell.kpts[ik], _dev(cell.gvecs[ik]))
    Ag, Bg = A.cpu().numpy().T, B.cpu().numpy().T
    if which == "c1":
        cols = np.sort(np.random.default_rng(1).choice(cell.n_g(ik), 200, replace=False))
        Ao, Bo = oracle_lib.coeffs(cell, ik, cols)
        Ag, Bg = Ag[:, cols], Bg[:, cols]
    else:
        Ao, Bo = oracle_lib.coeffs(cell, ik)
    for g, o in ((Ag, Ao), (Bg, Bo)):
        assert np.abs(g - o).max() <= 1e-13 * np.abs(o).max()
        # relative check where the entry is not the result of cancellation in the radial factor
        big = np.abs(o) > 1e-3 * np.abs(o).max()
        assert (np.abs(g - o)[big] / np.abs(o)[big]).max() < 1e-12


def test_coeffs_gamma_point(ctx, oracle_lib):
    cell = synthcells.custom_cell("gamma", 8.0, np.array([[0.5, 1.0, 2.0], [3.0, 1.0, 0.2]]),
                                  np.array([0, 0], np.int32), [6], [2.0], 2, 33, [5], kpts=np.zeros((1, 3)))
    A, B = ctx.coeffs(cell, cell.kpts[0], _dev(cell.gvecs[0]))
    Ao, Bo = oracle_lib.coeffs(cell, 0)
    assert np.abs(A.cpu().numpy().T - Ao).max() <= 1e-13 * np.abs(Ao).max()
    assert np.abs(B.cpu().numpy().T - Bo).max() <= 1e-13 * np.abs(Bo).max()


@pytest.mark.parametrize("which", ["c0", "mixed", "c2"])
def test_tmat_parity(ctx, oracle_lib, which):
    cell = {"c0": lambda: synthcells.config(0), "mixed": _mixed, "c2": lambda: synthcells.config(2)}[which]()
    T = ctx.build_T(cell).cpu().numpy()
    To = oracle_lib.tmat_all(cell)
    for ty in range(cell.n_types):
        Tg = T[ty].T                                  # stored column-major
        assert np.abs(Tg - To[ty]).max() <= 1e-13 * np.abs(To[ty]).max()


def test_hs_contract_random_operands(ctx, oracle_lib):
    """The contraction stage alone on non-coefficient-shaped operands (random A, B)."""
    cell = _mixed(n_g=300)
    A, B = synthcells.random_contraction_inputs([7, 7], cell.k_rows(), 300)
    T = ctx.build_T(cell)
    H, S = ctx.hs_contract(cell, _dev(A.T), _dev(B.T), T)
    Ho, So = oracle_lib.hs_block(cell, oracle_lib.tmat_all(cell), A, B, A, B)
    Hg, Sg = _upper(H.cpu().numpy()), _upper(S.cpu().numpy())
    assert _rel_err(Hg, Ho) < TOL_FP64
    assert _rel_err(Sg, So) < TOL_FP64


@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_hs_generate_full(ctx, oracle_lib, which):
    import torch
    cell = synthcells.config(0) if which == "c0" else _mixed()
    n = cell.n_g(0)
    sentinel = complex(7.0, -3.0)
    H = torch.full((n, n + 3), sentinel, dtype=torch.complex128, device="cuda")
    S = torch.full((n, n + 3), sentinel, dtype=torch.complex128, device="cuda")
    ctx.hs_generate(cell, cell.kpts, [_dev(cell.gvecs[0])], out=[(H, S)])
    Hn, Sn = H.cpu().numpy(), S.cpu().numpy()
    Ho, So = oracle_lib.hs_full(cell, 0)
    for M, R in ((Hn, Ho), (Sn, So)):
        full = _upper(M[:, :n])
        assert _rel_err(full, R) < TOL_FP64
        assert np.all(np.diag(M[:, :n]).imag == 0.0)
        low = np.tril(np.ones((n, n), bool), -1).T              # M[t, r] with r > t: lower part
        assert np.all(M[:, :n][low] == sentinel)
        assert np.all(M[:, n:] == sentinel)


def test_hs_generate_batched_mixed_lmax(ctx, oracle_lib):
    """Several k-points with different N_G and atom types with different l_max in one call;
    each k-point equals the oracle."""
    cell = _mixed(seed=21, n_g=190, n_k=3)
    out = ctx.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs])
    for ik, (H, S) in enumerate(out):
        Ho, So = oracle_lib.hs_full(cell, ik)
        assert _rel_err(_upper(H.cpu().numpy()), Ho) < TOL_FP64
        assert _rel_err(_upper(S.cpu().numpy()), So) < TOL_FP64


def test_hs_generate_batch_equals_single(ctx):
    cell = _mixed(seed=23, n_g=150, n_k=3)
    out = ctx.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs])
    for ik in range(3):
        H1, S1 = ctx.hs_generate(cell, cell.kpts[ik:ik + 1], [_dev(cell.gvecs[ik])])[0]
        assert np.array_equal(H1.cpu().numpy(), out[ik][0].cpu().numpy())
        assert np.array_equal(S1.cpu().numpy(), out[ik][1].cpu().numpy())


def _sampled_check(ctx, oracle_lib, cell, prec, tol, nsamp=48, slices=0):
    out = ctx.hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs], prec=prec, slices=slices)
    T = oracle_lib.tmat_all(cell)
    errs = []
    for ik, (H, S) in enumerate(out):
        n = cell.n_g(ik)
        rng = np.random.default_rng(100 + ik)
        idx = np.unique(np.concatenate([rng.choice(n, nsamp, replace=False), [0, n - 1]]))
        Ho, So = oracle_lib.hs_sampled(cell, ik, idx, idx, T)
        Hn, Sn = H.cpu().numpy(), S.cpu().numpy()
        up = idx[:, None] <= idx[None, :]
        for M, R in ((Hn, Ho), (Sn, So)):
            got = M[np.ix_(idx, idx)].T                          # entry (r, c) at M[c, r]
            e = float(np.linalg.norm((got - R)[up]) / np.linalg.norm(R[up]))
            errs.append(e)
            assert e < tol, (ik, e)
    return errs


def test_hs_generate_c1_sampled(ctx, oracle_lib):
    _sampled_check(ctx, oracle_lib, synthcells.config(1), "fp64", TOL_FP64)


def test_hs_generate_c3_subset_sampled(ctx, oracle_lib):
    """Batched workload shape: 4 of the 64 k-points (uneven N_G), sampled entries."""
    _sampled_check(ctx, oracle_lib, synthcells.config(3, n_k=4), "fp64", TOL_FP64, nsamp=32)
