"""bench.py host logic, on the CPU: the refusal of more than one GPU, the refusal without a GPU,
the default paths and step caps, the unbiased full-matrix error estimate, the counter-summary
lookup that fills the roofline's traffic (and its invalidation when the kernel source changes),
and the executed-operation factors of the split paths."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_no_gpu_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "no GPU" in r.stderr


def test_source_hash_is_the_kernel_file_hash():
    path = os.path.join(ROOT, "paper_1602_06589_amd", "csrc", "mod_contract.hip")
    with open(path, "rb") as f:
        assert bench.kernel_sources_sha("i8mod") == hashlib.sha256(f.read()).hexdigest()[:16]


def test_traffic_line_is_read_for_the_current_source(tmp_path, monkeypatch):
    sha = bench.kernel_sources_sha("i8mod")
    p = tmp_path / "traffic.txt"
    p.write_text("notes\n"
                 f"traffic kernel=hs_mod workload=c4_scale src_sha={sha} slices=11 bytes_per_launch=123000\n"
                 "traffic kernel=hs_mod workload=c1_realistic src_sha=0000000000000000 bytes_per_launch=7\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.read_traffic("i8mod", "c4_scale", 11) == 123000.0
    assert bench.read_traffic("i8mod", "c4_scale", 10) is None           # counters of another modulus count
    # a line recorded for another source version is ignored
    assert bench.read_traffic("i8mod", "c1_realistic") is None
    # other kernels and workloads without a line
    assert bench.read_traffic("fp64", "c4_scale") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic("i8mod", "c4_scale", 11) is None


@pytest.mark.parametrize("prec,slices,factor", [("i8mod", 10, 5.0), ("i8mod", 11, 5.5), ("i8", 6, 21.0),
                                                ("bf16", 6, 21.0), ("i8", 3, 6.0)])
def test_executed_operations_per_flop(prec, slices, factor):
    """Two real int8 products per modulus (half of a complex product's four); s(s+1)/2 digit-pair
    products of four real ones each for the digit schemes."""
    assert bench.executed_per_flop(slices, prec) == factor


def test_default_paths_and_step_caps():
    """Default run: the modular split headline and the FP64 comparator only, no matrix-core probe;
    the headline takes the requested steps, every other path at most 1 warm-up and 3 timed steps."""
    a = bench.make_parser().parse_args([])
    assert a.precs == "i8mod,fp64" and a.config == 4 and a.gpus == 1
    assert not a.ceiling and not a.eager
    assert a.steps >= 10 and a.warmup >= 3
    assert bench.step_plan(True, 20, 5) == (5, 20, 3)
    assert bench.step_plan(False, 20, 5) == (1, 3, 1)
    assert bench.step_plan(False, 2, 0) == (0, 2, 1)
    assert bench.step_plan(True, 1, 0) == (0, 1, 1)


def test_error_estimate_reweights_the_sample():
    """A random principal submatrix of n of N indices: the estimate weighs its diagonal by N/n and
    its pairs by N(N-1)/(n(n-1)); on a matrix whose error and value are uniform per class (diagonal,
    off-diagonal) it returns the whole matrix's relative Frobenius error exactly."""
    import numpy as np
    n, N = 50, 2000
    ref = np.full((n, n), 0.01, complex)
    np.fill_diagonal(ref, 1.0)
    err = np.full((n, n), 1e-12, complex)
    np.fill_diagonal(err, 1e-13)
    got = np.triu(ref + err)
    e = bench.error_estimates(got, np.triu(ref), N)
    full_err2 = N * 1e-26 + N * (N - 1) * 1e-24
    full_ref2 = N * 1.0 + N * (N - 1) * 1e-4
    assert abs(e["full_relF_est"] - np.sqrt(full_err2 / full_ref2)) < 1e-5 * e["full_relF_est"]   # rounding of ref + err
    # the sample's own error under-weights the off-diagonal error: the estimate is larger here
    assert e["full_relF_est"] > 2 * e["sample_relF"]
    assert abs(e["max_err_over_max"] - 1e-12) < 1e-17
    # a sample that is the whole matrix gives its own (Hermitian, full) error
    e2 = bench.error_estimates(got, np.triu(ref), n)
    full = lambda U: U + np.triu(U, 1).conj().T
    direct = np.linalg.norm(full(got) - ref) / np.linalg.norm(ref)
    assert abs(e2["full_relF_est"] - direct) < 1e-9 * direct


def test_mod_copy_bytes_counts_the_blocks_of_both_triangles():
    """N = 11621 spans 91 tiles of 128 columns (the 92nd, padding only, gets no block): 2116 blocks
    of 256 x 128 with 2I <= J per matrix, each copying 24 KB per 32-row group for every modulus."""
    assert bench.mod_copy_bytes(11621, 123904, 11) == 2 * 11 * 2116 * (123904 // 32) * 24576
    assert bench.mod_copy_bytes(11520, 128, 11) == 2 * 11 * 2070 * 4 * 24576      # 90 tiles, no padding tile
    assert bench.mod_copy_bytes(256, 256, 8) == 2 * 8 * 2 * 8 * 24576
    assert bench.mod_copy_bytes(129, 32, 8) == 2 * 8 * 2 * 1 * 24576


def test_contraction_rows_of_a_structured_t():
    """With S by the addition theorem and l_nonsph = 6, an l_max 10 atom contributes 49 rows of A
    instead of 121; an l_max 4 atom keeps its 25; without a structured T all rows count."""
    assert bench.contraction_rows([10, 10, 4], 6) == 49 + 49 + 25
    assert bench.contraction_rows([10, 10, 4], -1) == 121 + 121 + 25
