"""GPU parity of the interstitial terms and of the generalized eigensolve (section 2.3: eqs.
basis_function and HS_Mat over the cell minus the muffin-tin spheres; eq. matrix_kohnsham).

  * flapw_interstitial against the oracle's interstitial block: the whole matrix of the 2-atom
    workload (spheres moved apart) and of the 64-atom workload, sampled entries of the 512-atom
    workload; per entry within 1e-13 of the largest entry;
  * generation with the interstitial terms on equals the muffin-tin generation plus
    flapw_interstitial bit for bit (eager and HIP-graph replay), and the oracle's full H and S;
  * flapw_eigensolve on the full FP64 H and S of the 2- and 64-atom workloads: eigenvalues against
    the oracle's (scipy) eigenvalues of the oracle's matrices, eigenvectors by their residual and
    S-orthonormality in the oracle's matrices; the modular split H and S give eigenvalues within
    the error their 1e-10 relative matrix error allows;
  * the muffin-tin S alone (rank <= 2K < N) is refused as not positive definite."""
import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu
V_INT = 0.1


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


def _upper(M):
    U = np.triu(M.T)
    return U + np.triu(U, 1).conj().T


def _zeros(n):
    import torch
    return torch.zeros((n, n), dtype=torch.complex128, device="cuda")


def _check(got, ref, tol):
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("cfg", [0, 1])
def test_interstitial_full_matrix(ctx, oracle_lib, cfg):
    cell = synthcells.config_separated(cfg)
    n = cell.n_g(0)
    H, S = _zeros(n), _zeros(n)
    ctx.interstitial(cell, cell.kpts[0], _dev(cell.gvecs[0]), H, S, v_int=V_INT)
    Ho, So = oracle_lib.interstitial_block(cell, 0, v_int=V_INT)
    _check(_upper(S.cpu().numpy()), So, 1e-13)
    _check(_upper(H.cpu().numpy()), Ho, 1e-13)
    assert np.all(np.tril(S.cpu().numpy().T, -1) == 0)              # strictly lower part untouched


def test_interstitial_sampled_512_atoms(ctx, oracle_lib):
    """k-point 0 of the 512-atom workload (N = 11621): every 64-column tile row and column holds a
    sampled index; entries compared as an upper-triangle block."""
    cell = synthcells.config(4, n_k=1)
    n = cell.n_g(0)
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([np.arange(0, n, 64) + rng.integers(0, 64, size=(n + 63) // 64)]).clip(0, n - 1))
    H, S = _zeros(n), _zeros(n)
    ctx.interstitial(cell, cell.kpts[0], _dev(cell.gvecs[0]), H, S, v_int=V_INT)
    Ho, So = oracle_lib.interstitial_block(cell, 0, idx, idx, v_int=V_INT)
    up = idx[:, None] <= idx[None, :]
    for M, R in ((S, So), (H, Ho)):
        got = M.cpu().numpy()[np.ix_(idx, idx)].T                 # [row][col] = entry (idx_r, idx_c)
        assert np.abs(got - R)[up].max() <= 1e-13 * np.abs(R[up]).max()


@pytest.mark.parametrize("prec", ["fp64", "i8mod"])
def test_generation_with_interstitial(ctx, oracle_lib, prec):
    from paper_1602_06589_amd import Flapw
    import torch
    cell = synthcells.config_separated(0)
    g = [_dev(cell.gvecs[0])]
    n = cell.n_g(0)
    with Flapw() as f:
        (Hm, Sm), = f.hs_generate(cell, cell.kpts, g, prec=prec)
        f.interstitial(cell, cell.kpts[0], g[0], Hm, Sm, v_int=V_INT)
        f.set_interstitial(True, cell.lattice, V_INT)
        (Ht, St), = f.hs_generate(cell, cell.kpts, g, prec=prec)
        up = np.triu(np.ones((n, n), bool)).T
        assert np.array_equal(Ht.cpu().numpy()[up], Hm.cpu().numpy()[up])
        assert np.array_equal(St.cpu().numpy()[up], Sm.cpu().numpy()[up])
        with f.plan(cell, cell.kpts, g, prec=prec) as plan:
            for _ in range(2):
                for M in plan.out[0]:
                    M.fill_(complex(5.0, 5.0))
                plan.launch()
                torch.cuda.synchronize()
                assert np.array_equal(plan.out[0][0].cpu().numpy()[up], Hm.cpu().numpy()[up])
                assert np.array_equal(plan.out[0][1].cpu().numpy()[up], Sm.cpu().numpy()[up])
    Ho, So = oracle_lib.hs_total(cell, 0, v_int=V_INT)
    tol = 1e-12 if prec == "fp64" else 1e-10
    for got, ref in ((Ht, Ho), (St, So)):
        G = _upper(got.cpu().numpy())
        assert np.linalg.norm(G - ref) / np.linalg.norm(ref) < tol


@pytest.fixture(scope="module")
def oracle_total():
    import oracle
    out = {}
    for cfg in (0, 1):
        cell = synthcells.config_separated(cfg)
        H, S = oracle.hs_total(cell, 0, v_int=V_INT)
        w, C = oracle.eigh_generalized(H, S)
        out[cfg] = (cell, H, S, w)
    return out


@pytest.mark.parametrize("cfg", [0, 1])
def test_eigensolve(ctx, oracle_total, cfg):
    cell, Ho, So, wo = oracle_total[cfg]
    n = cell.n_g(0)
    g = [_dev(cell.gvecs[0])]
    ctx.set_interstitial(True, cell.lattice, V_INT)
    try:
        (H, S), = ctx.hs_generate(cell, cell.kpts, g, prec="fp64")
    finally:
        ctx.set_interstitial(False)
    w, C = ctx.eigensolve(H, S)
    w = w.cpu().numpy()
    C = C.cpu().numpy().T                                          # columns = eigenvectors
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wo).max() <= 1e-10 * np.abs(wo).max()
    scale = np.abs(Ho).max()
    R = Ho @ C - (So @ C) * w[None, :]
    assert np.abs(R).max() <= 1e-9 * scale * np.abs(C).max()
    assert np.abs(C.conj().T @ So @ C - np.eye(n)).max() <= 1e-9


def test_eigensolve_split_precision(ctx, oracle_total):
    """The modular split H and S (relative error <= 1e-10) move the eigenvalues by at most about
    cond(S) times that error."""
    cell, Ho, So, wo = oracle_total[1]
    g = [_dev(cell.gvecs[0])]
    ctx.set_interstitial(True, cell.lattice, V_INT)
    try:
        (H, S), = ctx.hs_generate(cell, cell.kpts, g, prec="i8mod")
    finally:
        ctx.set_interstitial(False)
    w, _ = ctx.eigensolve(H, S, vectors=False)
    cond = np.linalg.cond(So)
    assert np.abs(w.cpu().numpy() - wo).max() <= 1e-10 * cond * np.abs(wo).max()


def test_eigensolve_refuses_the_muffin_tin_overlap_alone(ctx):
    from paper_1602_06589_amd import FlapwError
    cell = synthcells.config_separated(0)
    assert cell.n_g(0) > 2 * cell.k_rows()
    (H, S), = ctx.hs_generate(cell, cell.kpts, [_dev(cell.gvecs[0])], prec="fp64")
    with pytest.raises(FlapwError) as ei:
        ctx.eigensolve(H, S)
    assert ei.value.status == -7
