"""Randomised GPU parity: seeded random cells (1-3 atom types with l_max 1-8, 2-7 atoms, random
positions, rotations and k-point, 40-420 basis functions) through the FP64 path and the modular
split with a random modulus count in 8..14, full H and S against the oracle.

Bars: FP64 1e-12; modular 2^(10 - B) with B the integer width of the count (the same bar as the
moduli test), and 1e-10 from 11 moduli on.  Each case prints its seed first."""
import math

import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu


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


def _rel_err(got, ref):
    e = float(np.abs(got - ref).max() / np.abs(ref).max())
    return max(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), e)


def _bits(nm):
    mods, c = [], 255
    while len(mods) < nm:
        if any((x * x + 1) % c == 0 for x in range(1, c)) and all(math.gcd(c, m) == 1 for m in mods):
            mods.append(c)
        c -= 2
    return min(50, int(math.floor((sum(math.log2(m) for m in mods) - 1) / 2)))


def _random_cell(seed):
    rng = np.random.default_rng(9000 + seed)
    n_types = int(rng.integers(1, 4))
    lmax = rng.integers(1, 9, size=n_types)
    rmt = rng.uniform(1.4, 2.2, size=n_types)
    n_atoms = int(rng.integers(2, 8))
    a = 10.0 + 2.0 * n_atoms
    pos = rng.uniform(0.0, a, size=(n_atoms, 3))
    types = rng.integers(0, n_types, size=n_atoms).astype(np.int32)
    types[:n_types] = np.arange(n_types)                 # every type used
    n_g = int(rng.integers(40, 421))
    return synthcells.custom_cell(f"random{seed}", a, pos, types, lmax.tolist(), rmt.tolist(), 4, n_g, [seed],
                                  rotations="random"), int(rng.integers(8, 15))


@pytest.mark.parametrize("seed", range(12))
def test_random_cell(ctx, oracle_lib, seed):
    cell, nm = _random_cell(seed)
    print(f"random cell seed {seed}: {cell.n_atoms} atoms, l_max {cell.lmax.tolist()}, N {cell.n_g(0)}, "
          f"moduli {nm}", flush=True)
    g = [_dev(cell.gvecs[0])]
    Ho, So = oracle_lib.hs_full(cell, 0)
    for prec, slices in (("fp64", 0), ("i8mod", nm)):
        (H, S), = ctx.hs_generate(cell, cell.kpts, g, prec=prec, slices=slices)
        eh = _rel_err(_upper(H.cpu().numpy()), Ho)
        es = _rel_err(_upper(S.cpu().numpy()), So)
        if prec == "fp64":
            tol = 1e-12
        else:
            tol = 2.0 ** (10 - _bits(nm)) + 1e-14
            if nm >= 11:
                tol = min(tol, 1e-10)
        assert eh < tol and es < tol, (seed, prec, slices, eh, es, tol)
