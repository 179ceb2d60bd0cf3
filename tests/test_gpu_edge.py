"""Edge cases of the whole path on the GPU, every precision and both S methods, against the
oracle: one basis function, exactly one tile and one tile plus one column (64, 128, 256), a single atom with
l_max and l''_max at the library caps, atoms with l_max 0 and 1, the Gamma point (K = 0 in the basis), and the largest
workload (c4_scale, k-point 0, in the configuration the benchmark times) on sampled entries.  All
four k-points of that workload: test_gpu_c4_batches.py."""
import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "i8": 1e-10, "bf16": 1e-10, "i8mod": 1e-10}


@pytest.fixture(scope="module")
def handles():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_06589_amd import Flapw
    g, l = Flapw(), Flapw()
    l.set_s_method("legendre")
    yield {"gemm": g, "legendre": l}
    g.close()
    l.close()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _upper(M):
    U = np.triu(M.T)
    return U + np.triu(U, 1).conj().T


def _relfro(got, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got))


def _rel_err(got, ref):
    """The larger of the relative Frobenius error and the largest entry error relative to the
    largest entry: a bound on either alone would let the other slip."""
    e = float(np.abs(got - ref).max() / np.abs(ref).max()) if np.abs(ref).max() > 0 else float(np.abs(got).max())
    return max(_relfro(got, ref), e)



def _cell(n_g, types=(0, 1, 0), lmax=(4, 6), lpot=4, seed=3, a=9.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, a, size=(len(types), 3))
    rmt = [1.6 + 0.1 * i for i in range(len(lmax))]
    return synthcells.custom_cell("edge", a, pos, np.array(types, np.int32), list(lmax), rmt, lpot, n_g, [seed],
                                  rotations="random")


def _check_full(handles, oracle_lib, cell, prec, method):
    out = handles[method].hs_generate(cell, cell.kpts, [_dev(g) for g in cell.gvecs], prec=prec)
    for ik, (H, S) in enumerate(out):
        Ho, So = oracle_lib.hs_full(cell, ik)
        eh = _rel_err(_upper(H.cpu().numpy()), Ho)
        es = _rel_err(_upper(S.cpu().numpy()), So)
        tol_s = 1e-12 if method == "legendre" else TOL[prec]
        assert eh < TOL[prec] and es < tol_s, (prec, method, ik, eh, es)
        assert np.all(np.diag(H.cpu().numpy()).imag == 0.0) and np.all(np.diag(S.cpu().numpy()).imag == 0.0)


@pytest.mark.parametrize("method", ["gemm", "legendre"])
@pytest.mark.parametrize("prec", ["fp64", "i8", "bf16", "i8mod"])
@pytest.mark.parametrize("n_g", [1, 64, 65, 128, 129, 256, 257])
def test_tile_edges(handles, oracle_lib, n_g, prec, method):
    """Tile boundaries: 64 (FP64 and digit tiles), 128 (modular reconstruction tiles) and 256
    (modular contraction blocks), each exactly and plus one column."""
    _check_full(handles, oracle_lib, _cell(n_g), prec, method)


@pytest.mark.parametrize("method", ["gemm", "legendre"])
@pytest.mark.parametrize("prec", ["fp64", "i8", "bf16", "i8mod"])
def test_caps_single_atom(handles, oracle_lib, prec, method):
    """One atom, l_max = 12 (2 NL = 338 rows) and l''_max = 12."""
    cell = _cell(230, types=(0,), lmax=(12,), lpot=12, seed=8, a=7.0)
    _check_full(handles, oracle_lib, cell, prec, method)


@pytest.mark.parametrize("method", ["gemm", "legendre"])
@pytest.mark.parametrize("prec", ["fp64", "i8", "bf16", "i8mod"])
def test_mixed_row_tiles(handles, oracle_lib, prec, method):
    """l_max 12 and 5 (2 NL = 338 and 72): the Q panels take two 256-row tiles, and the second
    tile of the l_max 5 atoms holds no rows (zero column-sum shares for the modular scaling)."""
    cell = _cell(170, types=(0, 1, 1), lmax=(12, 5), lpot=6, seed=23, a=8.0)
    _check_full(handles, oracle_lib, cell, prec, method)


@pytest.mark.parametrize("method", ["gemm", "legendre"])
@pytest.mark.parametrize("prec", ["fp64", "i8", "bf16", "i8mod"])
def test_smallest_lmax(handles, oracle_lib, prec, method):
    """Atoms with l_max 0 and 1 (2NL = 2 and 8 rows): most Q-panel waves hold no rows."""
    cell = _cell(150, types=(0, 1, 1, 0), lmax=(0, 1), lpot=2, seed=17)
    _check_full(handles, oracle_lib, cell, prec, method)


@pytest.mark.parametrize("method", ["gemm", "legendre"])
@pytest.mark.parametrize("prec", ["fp64", "i8", "bf16", "i8mod"])
def test_gamma_point(handles, oracle_lib, prec, method):
    """k = 0: the basis includes K = 0, whose direction is undefined (only l = 0 survives there)."""
    rng = np.random.default_rng(13)
    cell = synthcells.custom_cell("gamma", 9.0, rng.uniform(0, 9.0, size=(3, 3)), np.array([0, 1, 0], np.int32),
                                  [5, 3], [1.7, 1.9], 4, 97, [13], kpts=np.zeros((1, 3)), rotations="random")
    assert np.min(np.linalg.norm(cell.gvecs[0], axis=1)) == 0.0
    _check_full(handles, oracle_lib, cell, prec, method)


def test_c4_kpoint0_sampled(handles, oracle_lib):
    """The largest workload at full size (k-point 0: 512 atoms, K = 61952, N = 11621), the
    launch configuration of the benchmark, on 40 sampled basis functions plus the first and last.
    The modular path runs with the default 11 moduli (also the count the autotuner picks for this
    workload, the benchmark's) and with 12."""
    import torch
    cell = synthcells.config(4, n_k=1)
    g = [_dev(x) for x in cell.gvecs]
    n = cell.n_g(0)
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1]]))
    Ho, So = oracle_lib.hs_sampled(cell, 0, idx, idx, oracle_lib.tmat_all(cell))
    up = idx[:, None] <= idx[None, :]
    for method in ("gemm", "legendre"):
        for prec, slices in (("i8mod", 0), ("i8mod", 12), ("i8", 0), ("fp64", 0)):
            print(f"c4 k-point 0 sampled: {method} {prec} slices {slices}", flush=True)
            (H, S), = handles[method].hs_generate(cell, cell.kpts, g, prec=prec, slices=slices)
            sub_idx = _dev(idx)
            Hs = H[sub_idx][:, sub_idx].cpu().numpy().T      # entry (r, t) of the sample block
            Ss = S[sub_idx][:, sub_idx].cpu().numpy().T
            del H, S
            # one k-point of this size holds 100-160 GB of work buffers: free them before the next
            # path (the other handle's generation would not fit beside them)
            handles[method].release_workspace()
            torch.cuda.empty_cache()
            for name, got, ref in (("H", Hs, Ho), ("S", Ss, So)):
                err = float(np.linalg.norm((got - ref)[up]) / np.linalg.norm(ref[up]))
                tol = 1e-12 if (prec == "fp64" or (name == "S" and method == "legendre")) else 1e-10
                assert err < tol, (method, prec, slices, name, err)
