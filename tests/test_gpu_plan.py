"""GPU checks of the captured generation (HIP graph replay) and of the autotuner.

Replays: every replay of a plan must reproduce the eager flapw_hs_generate output bit for bit
(the same kernels run in the same order), with unrelated eager work and synchronisations between
replays and the outputs overwritten before each replay, and must meet the oracle bar.
Autotuner: the digit count it picks meets the tolerance it was given, and later calls with
slices = 0 use it."""
import math
import os

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


def _mixed(seed=31, n_g=190, n_k=2):
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



def _upper_mask(n):
    return np.triu(np.ones((n, n), bool)).T            # [t][r] with r <= t


def _replay_check(ctx, oracle_lib, cell, prec, tol, fraction=None):
    import torch
    g = [_dev(x) for x in cell.gvecs]
    old = os.environ.get("FLAPW_WORK_FRACTION")
    if fraction is not None:
        os.environ["FLAPW_WORK_FRACTION"] = fraction
    try:
        eager = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec=prec)]
        plan = ctx.plan(cell, cell.kpts, g, prec=prec)
    finally:
        if fraction is not None:
            if old is None:
                del os.environ["FLAPW_WORK_FRACTION"]
            else:
                os.environ["FLAPW_WORK_FRACTION"] = old
    other = _mixed(seed=5, n_g=150, n_k=1)
    other_g = [_dev(x) for x in other.gvecs]
    with plan:
        for rep in range(3):
            for H, S in plan.out:
                H.fill_(complex(float("nan"), 1.0))
                S.fill_(complex(-7.0, float("nan")))
            plan.launch()
            torch.cuda.synchronize()
            for ik, ((H, S), (He, Se)) in enumerate(zip(plan.out, eager)):
                up = _upper_mask(cell.n_g(ik))
                for got, ref in ((H.cpu().numpy(), He), (S.cpu().numpy(), Se)):
                    assert np.array_equal(got[up], ref[up]), (prec, rep, ik)
                    assert np.all(np.isnan(got[~up])), (prec, rep, ik)      # strictly lower part untouched
            ctx.hs_generate(other, other.kpts, other_g, prec="fp64")     # eager work between replays
            torch.cuda.synchronize()
        for ik, (H, S) in enumerate(plan.out):
            Ho, So = oracle_lib.hs_full(cell, ik)
            assert _rel_err(_upper(H.cpu().numpy()), Ho) < tol
            assert _rel_err(_upper(S.cpu().numpy()), So) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("i8", 1e-10), ("i8mod", 1e-10)])
def test_plan_replays_match_eager(ctx, oracle_lib, prec, tol):
    _replay_check(ctx, oracle_lib, _mixed(), prec, tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("i8", 1e-10), ("i8mod", 1e-10)])
def test_plan_one_kpoint_per_batch(ctx, oracle_lib, prec, tol):
    """A tiny work budget forces one memory batch per k-point (panels and digits reused)."""
    _replay_check(ctx, oracle_lib, _mixed(seed=8, n_g=130, n_k=3), prec, tol, fraction="1e-12")


def test_eager_one_kpoint_per_batch_equals_grouped(ctx):
    cell = _mixed(seed=9, n_g=160, n_k=3)
    g = [_dev(x) for x in cell.gvecs]
    for prec in ("fp64", "i8", "i8mod"):
        grouped = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec=prec)]
        os.environ["FLAPW_WORK_FRACTION"] = "1e-12"
        try:
            single = [(H.cpu().numpy(), S.cpu().numpy()) for H, S in ctx.hs_generate(cell, cell.kpts, g, prec=prec)]
        finally:
            del os.environ["FLAPW_WORK_FRACTION"]
        for ik, ((a, b), (c, d)) in enumerate(zip(grouped, single)):
            up = _upper_mask(cell.n_g(ik))
            assert np.array_equal(a[up], c[up]) and np.array_equal(b[up], d[up]), (prec, ik)


def test_tune_digits_and_use(ctx, oracle_lib):
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=44, n_g=300, n_k=1)
    g = _dev(cell.gvecs[0])
    Ho, So = oracle_lib.hs_full(cell, 0)
    with Flapw() as f:
        for tol in (1e-10, 1e-6):
            res = f.tune(cell, cell.kpts[0], g, prec="i8", tol=tol)
            s = res["slices"]
            assert 3 <= s <= 6 and res["band"] in (1, 2, 4, 8, 16), res
            errs = res["digit_err"]
            assert all(math.isfinite(e) for e in errs)
            assert all(errs[i + 1] < errs[i] for i in range(3)), errs
            # n_g <= 1024: the tuner's sample is the whole matrix (extrapolation factor 1)
            assert errs[s - 3] <= 2 * tol / 3 and (s == 3 or errs[s - 4] > 2 * tol / 3), res
            assert all(math.isfinite(t) and t > 0 for t in res["band_ms"][:5]), res
            assert res["stage_rows"] == 0 and all(math.isnan(t) for t in res["band_ms"][5:]), res
            # slices = 0 now means the tuned count: bitwise equal to asking for it explicitly
            (H0, S0), = f.hs_generate(cell, cell.kpts, [g], prec="i8")
            (H1, S1), = f.hs_generate(cell, cell.kpts, [g], prec="i8", slices=s)
            up = _upper_mask(cell.n_g(0))
            assert np.array_equal(H0.cpu().numpy()[up], H1.cpu().numpy()[up])
            assert np.array_equal(S0.cpu().numpy()[up], S1.cpu().numpy()[up])
            assert _rel_err(_upper(H0.cpu().numpy()), Ho) < tol
            assert _rel_err(_upper(S0.cpu().numpy()), So) < tol
        assert res["slices"] < 6                                       # a loose tolerance needs fewer digits


def test_tune_fp64_and_unreachable(ctx):
    from paper_1602_06589_amd import FlapwError
    cell = _mixed(seed=45, n_g=200, n_k=1)
    g = _dev(cell.gvecs[0])
    res = ctx.tune(cell, cell.kpts[0], g, prec="fp64", tol=1e-12)
    assert res["slices"] == 0 and res["band"] in (1, 2, 4, 8, 16)
    assert all(math.isnan(e) for e in res["digit_err"])
    with pytest.raises(FlapwError) as ei:
        ctx.tune(cell, cell.kpts[0], g, prec="i8", tol=1e-30)
    assert ei.value.status == -6
    assert all(math.isfinite(e) for e in ei.value.result["digit_err"])


def test_tune_moduli_and_use(ctx, oracle_lib):
    """Modular split: the tuner picks the smallest of 10..13 moduli meeting 2 tol / 3."""
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=46, n_g=300, n_k=1)
    g = _dev(cell.gvecs[0])
    Ho, So = oracle_lib.hs_full(cell, 0)
    with Flapw() as f:
        res = f.tune(cell, cell.kpts[0], g, prec="i8mod", tol=1e-10)
        s = res["slices"]
        errs = res["digit_err"]
        assert 10 <= s <= 13 and res["band"] in (1, 2, 4, 8, 16), res
        assert res["stage_rows"] in (32, 64) and all(math.isfinite(t) and t > 0 for t in res["band_ms"]), res
        assert all(math.isfinite(e) for e in errs)
        assert errs[s - 10] <= 2e-10 / 3 and (s == 10 or errs[s - 11] > 2e-10 / 3), res
        assert all(errs[i + 1] < errs[i] for i in range(2)), errs
        (H0, S0), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod")
        (H1, S1), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod", slices=s)
        up = _upper_mask(cell.n_g(0))
        assert np.array_equal(H0.cpu().numpy()[up], H1.cpu().numpy()[up])
        assert np.array_equal(S0.cpu().numpy()[up], S1.cpu().numpy()[up])
        assert _rel_err(_upper(H0.cpu().numpy()), Ho) < 1e-10
        assert _rel_err(_upper(S0.cpu().numpy()), So) < 1e-10


def test_tuned_count_used_with_legendre_s_and_structured_t(ctx):
    """The tuner's choice is found again by generations under the same handle settings, also when S
    comes from the addition theorem and a structured T cuts the contraction rows (the layout the
    choice is keyed on is the cut one), and not under other settings."""
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=47, n_g=260, n_k=1)
    g = _dev(cell.gvecs[0])
    up = _upper_mask(cell.n_g(0))
    with Flapw() as f:
        f.set_s_method("legendre")
        f.set_lnonsph(2)
        res = f.tune(cell, cell.kpts[0], g, prec="i8mod", tol=1e-4)       # loose: the smallest candidate
        assert res["slices"] == 10, res
        (H0, _), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod")
        (H10, _), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod", slices=10)
        (H11, _), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod", slices=11)
        h0, h10, h11 = (x.cpu().numpy()[up] for x in (H0, H10, H11))
        assert np.array_equal(h0, h10)
        assert not np.array_equal(h0, h11)                               # 11 moduli: the default
        f.set_lnonsph(-1)                                                # another key: the default again
        f.set_s_method("gemm")
        (Hd, _), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod")
        (Hd11, _), = f.hs_generate(cell, cell.kpts, [g], prec="i8mod", slices=11)
        assert np.array_equal(Hd.cpu().numpy()[up], Hd11.cpu().numpy()[up])


def test_workspace_limit_releases_after_the_call(ctx):
    """With a workspace limit the handle frees its work buffers after a generation that leaves them
    above it (so that a second handle or the caller can allocate), and the results are unchanged."""
    from paper_1602_06589_amd import Flapw
    cell = _mixed(seed=48, n_g=333, n_k=2)
    g = [_dev(x) for x in cell.gvecs]
    with Flapw() as keep, Flapw() as trim:
        trim.set_workspace_limit(1 << 20)
        for prec in ("fp64", "i8mod"):
            a = keep.hs_generate(cell, cell.kpts, g, prec=prec)
            assert keep.workspace_bytes > (1 << 20)                 # kept for the next call
            b = trim.hs_generate(cell, cell.kpts, g, prec=prec)
            assert trim.workspace_bytes == 0, prec
            for ik, ((H0, S0), (H1, S1)) in enumerate(zip(a, b)):
                up = _upper_mask(cell.n_g(ik))
                assert np.array_equal(H0.cpu().numpy()[up], H1.cpu().numpy()[up])
                assert np.array_equal(S0.cpu().numpy()[up], S1.cpu().numpy()[up])
        trim.set_workspace_limit(-1)
        trim.hs_generate(cell, cell.kpts, g, prec="fp64")
        assert trim.workspace_bytes > 0
