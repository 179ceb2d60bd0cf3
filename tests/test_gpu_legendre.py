"""GPU parity of S through the addition theorem (section 3.1, eq. overlap_no_m with the prefactor
4 pi / Omega) against the FP64 oracle's S (its definition, eq. def_overlap), and of the
generation path that uses it (S by the addition theorem, H by the contraction).

Bar: relative Frobenius error <= 1e-12 (FP64 arithmetic throughout)."""
import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def _relfro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _rel_err(got, ref):
    """The larger of the relative Frobenius error and the largest entry error relative to the
    largest entry: a bound on either alone would let the other slip."""
    e = float(np.abs(got - ref).max() / np.abs(ref).max()) if np.abs(ref).max() > 0 else float(np.abs(got).max())
    return max(_relfro(got, ref), e)



def _mixed(seed=12, n_g=517, n_k=1, types=(0, 1, 0, 2, 1), lmax=(5, 3, 8), kpts=None):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 9.0, size=(len(types), 3))
    return synthcells.custom_cell("mixed", 9.0, pos, np.array(types, np.int32), list(lmax),
                                  [2.0, 1.7, 1.5, 1.9][:len(lmax)], 4, [n_g + 37 * i for i in range(n_k)], [seed],
                                  rotations="random", kpts=kpts)


@pytest.mark.parametrize("which", ["c0", "mixed"])
def test_s_legendre_full(ctx, oracle_lib, which):
    cell = synthcells.config(0) if which == "c0" else _mixed()
    S = ctx.s_legendre(cell, cell.kpts[0], _dev(cell.gvecs[0])).cpu().numpy()
    _, So = oracle_lib.hs_full(cell, 0)
    assert _rel_err(_upper(S), So) < TOL
    assert np.all(np.diag(S).imag == 0.0)


def test_s_legendre_gamma_and_empty_type(ctx, oracle_lib):
    """k = 0 with G = 0 in the list (K_0 = 0: only l = 0 survives), and a type without atoms."""
    cell = _mixed(seed=5, n_g=300, types=(0, 2, 0, 2), lmax=(4, 6, 7), kpts=np.zeros((1, 3)))
    assert np.min(np.linalg.norm(cell.gvecs[0], axis=1)) == 0.0
    S = ctx.s_legendre(cell, cell.kpts[0], _dev(cell.gvecs[0])).cpu().numpy()
    _, So = oracle_lib.hs_full(cell, 0)
    assert _rel_err(_upper(S), So) < TOL


def test_s_legendre_lower_untouched(ctx):
    import torch
    cell = _mixed(n_g=200)
    n = cell.n_g(0)
    S = torch.full((n, n + 3), complex(3.0, -1.0), dtype=torch.complex128, device="cuda")
    ctx.s_legendre(cell, cell.kpts[0], _dev(cell.gvecs[0]), S=S)
    M = S.cpu().numpy()
    low = np.tril(np.ones((n, n), bool), -1).T
    assert np.all(M[:, :n][low] == complex(3.0, -1.0)) and np.all(M[:, n:] == complex(3.0, -1.0))


def _sampled_S(cell, oracle_lib, S, ik, nsamp=40):
    n = cell.n_g(ik)
    rng = np.random.default_rng(300 + ik)
    idx = np.unique(np.concatenate([rng.choice(n, nsamp, replace=False), [0, n - 1]]))
    _, So = oracle_lib.hs_sampled(cell, ik, idx, idx, oracle_lib.tmat_all(cell))
    up = idx[:, None] <= idx[None, :]
    got = S[np.ix_(idx, idx)].T
    return float(np.linalg.norm((got - So)[up]) / np.linalg.norm(So[up]))


def test_s_legendre_c1_c2_sampled(ctx, oracle_lib):
    for i in (1, 2):
        cell = synthcells.config(i)
        S = ctx.s_legendre(cell, cell.kpts[0], _dev(cell.gvecs[0])).cpu().numpy()
        assert _sampled_S(cell, oracle_lib, S, 0) < TOL, i


@pytest.mark.parametrize("prec", ["fp64", "i8"])
def test_generate_with_legendre_S(ctx, oracle_lib, prec):
    """S from the addition theorem, H from the contraction: H equals the combined path's H bit
    for bit (same kernels and summation order), S meets the FP64 bar in both precisions."""
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=21, n_g=190, n_k=3)
    g = [_dev(x) for x in cell.gvecs]
    ref = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec=prec)]
    with Flapw() as f:
        f.set_s_method("legendre")
        out = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in f.hs_generate(cell, cell.kpts, g, prec=prec)]
        for ik, ((H, S), (Hr, _)) in enumerate(zip(out, ref)):
            up = np.triu(np.ones((cell.n_g(ik),) * 2, bool)).T
            assert np.array_equal(H[up], Hr[up]), ik
            _, So = oracle_lib.hs_full(cell, ik)
            assert _rel_err(_upper(S), So) < TOL, ik
        # the captured path replays the same thing
        with f.plan(cell, cell.kpts, g, prec=prec) as plan:
            for H, S in plan.out:
                H.fill_(0)
                S.fill_(0)
            for _ in range(2):
                plan.launch()
            for (H, S), (He, Se) in zip(plan.out, out):
                n = H.shape[0]
                up = np.triu(np.ones((n, n), bool)).T
                assert np.array_equal(H.cpu().numpy()[up], He[up]) and np.array_equal(S.cpu().numpy()[up], Se[up])
