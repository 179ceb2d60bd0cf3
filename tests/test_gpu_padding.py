"""Regression test: the padding rows of the work panels (between 2K and the 256-row alignment)
must not leak stale device memory into H and S.  The device allocator is first filled with NaN
patterns (through torch tensors that are then freed), then the library allocates its work
buffers; every path must still produce finite results equal to the oracle's."""
import numpy as np
import pytest

import synthcells

pytestmark = pytest.mark.gpu


def test_stale_memory_does_not_leak():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_06589_amd import Flapw
    import oracle
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 9.0, size=(5, 3))
    cell = synthcells.custom_cell("pad", 9.0, pos, np.array([0, 1, 0, 2, 1], np.int32), [5, 3, 8],
                                  [2.0, 1.7, 1.5], 4, 190, [3], rotations="random")
    assert (2 * cell.k_rows()) % 256 != 0                       # there are padding rows
    g = [torch.as_tensor(np.ascontiguousarray(cell.gvecs[0]), device="cuda")]
    Ho, So = oracle.hs_full(cell, 0)
    for prec, tol in (("fp64", 1e-12), ("i8", 1e-10), ("bf16", 1e-10), ("i8mod", 1e-10)):
        junk = torch.full((1 << 27,), float("nan"), dtype=torch.float64, device="cuda")   # 1 GiB of NaN
        del junk
        torch.cuda.empty_cache()
        with Flapw() as f:
            (H, S), = f.hs_generate(cell, cell.kpts, g, prec=prec)
            for M, R in ((H.cpu().numpy(), Ho), (S.cpu().numpy(), So)):
                U = np.triu(M.T)
                full = U + np.triu(U, 1).conj().T
                assert np.all(np.isfinite(full)), prec
                assert np.linalg.norm(full - R) / np.linalg.norm(R) < tol, prec
