#!/usr/bin/env python3
"""Benchmark: H and S generation (coefficients -> T -> per-atom panels -> S/H contractions) on
one MI355X, for the seeded synthetic workloads of synthcells (default: the 512-atom workload, 4
k-points).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--precs i8mod,fp64]
                    [--slices s | --no-tune] [--eager] [--ceiling] [--budget-s 420]

A path is a precision (i8mod, i8, bf16 or fp64 for the S/H contraction) with an optional "+leg": S
then comes from the addition theorem (section 3.1) and the contraction computes H alone.  The
first path is the headline; the default pair is the modular int8 split and the FP64 comparator.
Before its timing, each split path runs the library's autotuner on k-point 0 (flapw_tune: the
smallest modulus or digit count whose H and S errors, estimated for the whole matrix from a random
sample of basis functions, are at most 2/3 of 1e-10, then the fastest tile band and stage depth);
--slices fixes the count instead and --no-tune takes the defaults.
A step is one generation over every k-point of the workload (the whole path), replayed from a
HIP graph (flapw_plan_launch; --eager: flapw_hs_generate calls).  The headline takes W untimed
and K timed steps; every other path at most 1 and 3 (a wall-clock guard trims them further and
says so).  Each timed step lies between HIP events on the launch stream; the timed region is
bracketed by torch.cuda.synchronize().  G lists are resident in HBM before timing starts.
Prints one JSON line:
  value         algorithmic TFLOP/s of the headline from the median step time, F_alg per
                k-point = 16 K N(N+1) + 32 N sum_a NL_a^2 (S and H upper triangles + panels)
  ms_per_step   that median (mean, minimum and the host-clock mean beside it in "paths")
  roofline      the dominant kernel (the S/H contraction): its average launch time from the HIP
                events the library records on the launch stream during eager profiled steps
  rel_err       per matrix, the relative Frobenius error of the whole k-point-0 matrix estimated
                without bias from a random principal submatrix against the oracle
  cpu_baseline  the oracle timed on that sample, with the time of a whole k-point extrapolated
  radial_setup  radial functions and integral tables of the workload's atom types from synthetic
                meshes (--radial-nr points): GPU time per call, the oracle's time and deviation
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64": 78.6, "bf16": 2500.0, "i8": 5000.0, "i8mod": 5000.0}   # MI355X dense matrix-core peaks, T(FL)OP/s
# int8 (or bf16) operations the split kernel executes per algorithmic FP64 flop: 8 ops per complex
# multiply-add per digit pair (4 real products), s(s+1)/2 pairs, against 8 flops per complex
# multiply-add in the FP64 count; the modular path splits each complex product modulo a modulus
# into two real ones (4 ops per complex multiply-add)
def executed_per_flop(slices: int, prec: str = "i8") -> float:
    return slices / 2.0 if prec == "i8mod" else slices * (slices + 1) / 2.0
KERNEL = {"fp64": "hs_fp64", "bf16": "hs_split", "i8": "hs_split", "i8mod": "hs_mod"}
DEFAULT_SLICES = {"i8": 6, "bf16": 6, "i8mod": 11}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def kernel_sources_sha(prec: str) -> str:
    names = {"fp64": ["contract_fp64.hip"], "i8": ["split.hip"], "bf16": ["split_bf16.hip"],
             "i8mod": ["mod_contract.hip"]}[prec]
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1602_06589_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(prec: str, workload: str, slices: int = 0):
    """HBM bytes per launch of the contraction kernel from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken (or, for a line that names
    its digit or modulus count, when the count differs)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha = kernel_sources_sha(prec)
    for line in open(TRAFFIC_FILE):
        if not line.startswith("traffic "):
            continue
        kv = dict(x.split("=", 1) for x in line.split()[1:])
        if kv.get("kernel") == KERNEL[prec] and kv.get("workload") == workload and kv.get("src_sha") == sha \
                and ("slices" not in kv or int(kv["slices"]) == slices):
            return float(kv["bytes_per_launch"])
    return None


def oracle_threads() -> int:
    """Threads the oracle's OpenMP loops use (libgomp's own count), else the visible cores."""
    import ctypes
    try:
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def sample_indices(n: int, nsamp: int, seed: int = 4242) -> np.ndarray:
    """A uniform random subset of the basis functions of one k-point (sorted)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, min(nsamp, n), replace=False))


def gather_block(M, idx: np.ndarray) -> np.ndarray:
    """Entries (idx[a], idx[b]), a <= b, of an upper-triangle result tensor (M[c][r] = entry (r, c)),
    gathered on the device and copied to the host; the strictly lower part of the block is zero."""
    import torch
    ii = torch.as_tensor(idx, device=M.device)
    sub = M.index_select(0, ii).index_select(1, ii).transpose(0, 1).cpu().numpy()
    return np.triu(sub)


def error_estimates(got: np.ndarray, ref: np.ndarray, n_full: int) -> dict:
    """Errors of a result on the principal submatrix of a uniform random index sample.
    sample_relF: relative Frobenius error of the sample's upper triangle as it stands.
    full_relF_est: the same for the whole Hermitian matrix, from the sample reweighted so that the
    estimate of every squared norm is unbiased: the n sampled diagonal entries stand for the N
    diagonal entries (factor N/n), the n(n-1)/2 sampled pairs t' < t for the N(N-1)/2 pairs
    (factor N(N-1)/(n(n-1))), and the strict upper triangle counts twice (Hermitian).
    max_err_over_max: max |dX| over max |X| on the sample."""
    n = got.shape[0]
    iu = np.triu_indices(n, 1)
    d = np.arange(n)
    e2 = np.abs(got - ref) ** 2
    r2 = np.abs(ref) ** 2
    wd = n_full / n
    wo = n_full * (n_full - 1.0) / (n * (n - 1.0)) if n > 1 else 0.0
    num = wd * e2[d, d].sum() + 2.0 * wo * e2[iu].sum()
    den = wd * r2[d, d].sum() + 2.0 * wo * r2[iu].sum()
    up = np.triu(np.ones((n, n), bool))
    return {"sample_relF": float(np.sqrt(e2[up].sum() / r2[up].sum())),
            "full_relF_est": float(np.sqrt(num / den)),
            "max_err_over_max": float(np.sqrt(e2[up].max() / r2[up].max()))}


def cpu_baseline_leg(cell, idx: np.ndarray, lnonsph: int = -1):
    """The oracle on a bounded sample of k-point 0: H and S on the principal submatrix of the
    random basis-function subset idx (coefficients of those columns, T, per-atom panels, entries),
    timed on the host cores, plus a one-row block that isolates the per-column panel cost.  The
    time of a whole k-point is extrapolated from those parts (coefficients and panels per column,
    entries per upper-triangle entry) and labelled as such.  Returns (baseline, (H, S) of the
    sample)."""
    import oracle
    oracle._load()
    ik = 0
    n_full = cell.n_g(ik)
    ns = len(idx)
    t0 = time.perf_counter()
    T = oracle.tmat_all(cell, lnonsph=lnonsph)
    t_T = time.perf_counter() - t0
    t0 = time.perf_counter()
    A, B = oracle.coeffs(cell, ik, idx)
    t_coef = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ho, So = oracle.hs_block(cell, T, A, B, A, B)
    t_blk = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.hs_block(cell, T, A[:, :1], B[:, :1], A, B)          # one bra row: the panels of ns columns
    t_panel = time.perf_counter() - t0
    t_entry = max(t_blk - t_panel, 1e-9) / float(ns * ns)
    dt = t_T + t_coef + t_blk
    k = cell.k_rows()
    nl = cell.nl_atom().astype(float)
    flops = 32.0 * k * ns * ns + ns * 32.0 * float((nl * nl).sum())   # S and H entries + panels
    t_kpt = t_T + (t_coef + t_panel) * n_full / ns + t_entry * n_full * (n_full + 1) / 2.0
    base = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"k-point 0 of {cell.name}: H and S on the {ns}x{ns} principal submatrix of a random subset "
                      f"of its {n_full} basis functions (T, coefficients of those columns, per-atom panels, "
                      f"{ns * ns} entries), {dt:.1f} s",
            "seconds": dt,
            "seconds_per_kpoint_extrapolated": t_kpt,
            "extrapolation": f"T {t_T:.2f} s + (coefficients {t_coef:.2f} s + panels {t_panel:.2f} s) x N/{ns} + "
                             f"{t_entry * 1e6:.1f} us per entry x N(N+1)/2, N = {n_full}"}
    return base, (Ho, So)


def radial_leg(cell, n_r: int, steps: int, with_oracle: bool):
    """Radial functions and the four integral tables of the workload's atom types from synthetic
    meshes (one flapw_radial_setup call: upload, two kernels, download), timed on the GPU; with
    with_oracle also the oracle's time for the same call and the largest deviation from it."""
    import synthcells
    from paper_1602_06589_amd import Flapw
    m = synthcells.radial_meshes(cell.lmax, cell.rmt, cell.lpot, n_r=n_r, seed=0)
    with Flapw() as fl:
        got = fl.radial_setup(m.n_r, m.r0, m.rmt, m.v_sph, m.e_l, m.lmax, m.v_lm, m.lpot)
        fl.profile(True)
        t0 = time.perf_counter()
        for _ in range(max(1, steps)):
            got = fl.radial_setup(m.n_r, m.r0, m.rmt, m.v_sph, m.e_l, m.lmax, m.v_lm, m.lpot)
        call_ms = (time.perf_counter() - t0) * 1e3 / max(1, steps)
        n_l, k_ms = fl.kernel_time("radial")
        fl.profile(False)
    res = {"n_types": int(len(m.lmax)), "lmax": int(m.lmax.max()), "lpot": m.lpot, "n_r": n_r,
           "ms_per_call": call_ms, "kernels_ms_per_call": k_ms / max(1, n_l)}
    if with_oracle:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.radial_setup(m.n_r, m.r0, m.rmt, m.v_sph, m.e_l, m.lmax, m.v_lm, m.lpot)
        res["oracle_s"] = time.perf_counter() - t0
        res["max_err_rel_to_array_max"] = max(
            float(np.max(np.abs(got[k] - ref[k])) / np.max(np.abs(ref[k])))
            for k in ("u", "du", "ud", "dud", "ud_norm2", "i_uu", "i_ud", "i_du", "i_dd"))
    print(f"# radial setup: {json.dumps(res)}", flush=True)
    return res


def mfma_ceiling():
    """Matrix-core rates on register-resident operands distributed like the library's (the
    microbenchmark built next to the library), or None when it is not built."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1602_06589_amd", "mfma_rate")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def copy_ceiling():
    """L2 -> LDS copy rates (LDS-DMA and through registers), HBM -> LDS streaming and LDS read rates
    of the microbenchmark built next to the library, or None when it is not built."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1602_06589_amd", "copy_rate")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def contraction_rows(lmax_atoms, lnonsph: int) -> int:
    """Rows of A (or of B) the H contraction covers when S comes from the addition theorem: with a
    structured T (lnonsph >= 0) only the (min(l_max, lnonsph) + 1)^2 rows of each atom, the
    L-diagonal rest being added by the Legendre kernel; all K rows otherwise."""
    lm = np.asarray(lmax_atoms, dtype=np.int64)
    if lnonsph >= 0:
        lm = np.minimum(lm, lnonsph)
    return int(((lm + 1) ** 2).sum())


def mod_copy_bytes(n: int, kp2: int, nm: int) -> int:
    """Bytes the modular contraction copies from L2 into LDS for one k-point: every 256 x 128 block
    of the S and the H upper triangles (2I <= J over the ceil(N / 128) column tiles that hold
    columns), per modulus, copies 24 KB per 32-row group (256 + 128 columns x 2 evaluations x 32
    bytes)."""
    nt = (n + 127) // 128
    blocks = sum(nt - 2 * i for i in range((nt + 1) // 2))
    return 2 * nm * blocks * (kp2 // 32) * 24576


def step_plan(is_head: bool, steps: int, warmup: int):
    """(warm-up replays, timed replays, eager profiled steps) of a path: the headline takes the
    requested counts; every other path at most 1 warm-up and 3 timed replays, and one eager step
    for its kernel breakdown (the headline: up to 3, after one eager warm-up)."""
    if is_head:
        return warmup, steps, min(3, max(1, steps))
    return min(warmup, 1), min(steps, 3), 1


def operand_study(config: int, slices: int, reps: int = 2):
    """The modular contraction of one k-point-sized problem (the workload's atoms and K, its first
    k-point's N) through flapw_hs_contract on two operand sets of the same shape: seeded random
    complex A, B (residues spread over every int8 value) and constant A = B = 1 + i.  T is the
    identity and every ||udot||^2 is 1, so that P, d.P and Q are the same matrix and, in the constant
    case, every residue of a modulus is the same byte.  The instruction stream is identical; only the
    switching activity of the matrix-core operands differs, so a time difference shows a
    power-limited clock.  Returns the contraction kernel's average launch time (HIP events) per
    operand set."""
    import dataclasses
    import torch
    import synthcells
    from paper_1602_06589_amd import Flapw
    cell = synthcells.config(config, n_k=1)
    cell = dataclasses.replace(cell, ud_norm2=np.ones_like(cell.ud_norm2))
    n, kr = cell.n_g(0), cell.k_rows()
    gen = torch.Generator(device="cuda").manual_seed(1602)
    res = {"workload": cell.name, "K": kr, "n_g": n, "slices": slices}
    with Flapw() as fl:
        ldt = 2 * int((cell.lmax.max() + 1) ** 2)
        T = torch.eye(ldt, dtype=torch.complex128, device="cuda").repeat(cell.n_types, 1, 1).contiguous()
        H = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        S = torch.zeros_like(H)
        for kind in ("random", "constant"):
            if kind == "random":
                A = torch.randn((n, kr), dtype=torch.complex128, device="cuda", generator=gen)
                B = torch.randn((n, kr), dtype=torch.complex128, device="cuda", generator=gen)
            else:
                A = torch.full((n, kr), complex(1.0, 1.0), dtype=torch.complex128, device="cuda")
                B = torch.full_like(A, complex(1.0, 1.0))
            fl.hs_contract(cell, A, B, T, prec="i8mod", slices=slices, H=H, S=S)       # warm-up
            torch.cuda.synchronize()
            fl.profile(True)
            for _ in range(reps):
                fl.hs_contract(cell, A, B, T, prec="i8mod", slices=slices, H=H, S=S)
            torch.cuda.synchronize()
            nl, ms = fl.kernel_time("hs_mod")
            fl.profile(False)
            res[kind + "_ms"] = ms / max(1, nl)
            print(f"# operand study {kind}: hs_mod {ms / max(1, nl):.1f} ms per launch", flush=True)
            del A, B
            torch.cuda.empty_cache()
    res["random_over_constant"] = res["random_ms"] / res["constant_ms"]
    return res


def oracle_times(configs, one_core_max_n: int = 300, full_max_n: int = 3000, nsamp: int = 384):
    """The oracle's time per k-point for the named workloads, on the host cores: whole k-points
    (H and S of every basis-function pair, T, coefficients) up to full_max_n basis functions, and on
    one core (OMP_NUM_THREADS=1, a child process) up to one_core_max_n; larger k-points are
    extrapolated from a random principal submatrix as in the CPU baseline and labelled so."""
    import subprocess
    import synthcells
    import oracle
    oracle._load()
    out = []
    for c in configs:
        cell = synthcells.config(c, n_k=1)
        n = cell.n_g(0)
        rec = {"workload": cell.name, "n_g": n, "K": cell.k_rows(), "cores": oracle_threads()}
        if n <= full_max_n:
            t0 = time.perf_counter()
            oracle.hs_full(cell, 0)
            rec["seconds_full"] = time.perf_counter() - t0
        else:
            base, _ = cpu_baseline_leg(cell, sample_indices(n, nsamp))
            rec["seconds_extrapolated"] = base["seconds_per_kpoint_extrapolated"]
            rec["extrapolation"] = base["extrapolation"]
        if n <= one_core_max_n:
            code = (f"import sys, time; sys.path.insert(0, {ROOT!r}); import synthcells, oracle; "
                    f"cell = synthcells.config({c}, n_k=1); t0 = time.perf_counter(); oracle.hs_full(cell, 0); "
                    "print(time.perf_counter() - t0)")
            env = dict(os.environ, OMP_NUM_THREADS="1")
            r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=3600)
            rec["seconds_full_one_core"] = float(r.stdout.strip().splitlines()[-1])
        print(f"# oracle {json.dumps(rec)}", flush=True)
        out.append(rec)
    return out


def eigen_leg(config: int, prec: str, vectors: bool = True):
    """The generalized eigensolve of k-point 0 (full H and S: muffin tins plus the interstitial
    region with v_int = 0.1): generation time, flapw_eigensolve time (HIP events on the stream),
    and the lowest and highest eigenvalues."""
    import torch
    import synthcells
    from paper_1602_06589_amd import Flapw
    cell = synthcells.config_separated(config, n_k=1)
    g = [torch.as_tensor(np.ascontiguousarray(cell.gvecs[0]), device="cuda")]
    stream = torch.cuda.current_stream()
    res = {"workload": cell.name, "n_g": cell.n_g(0), "prec": prec, "vectors": vectors}
    def timed(fn):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), out

    with Flapw() as fl:
        fl.set_interstitial(True, cell.lattice, 0.1)
        (H, S), = fl.hs_generate(cell, cell.kpts, g, prec=prec)        # warm-up (allocations, tuning-free)
        # the first eigensolve also creates the solver's handle and workspace; it overwrites H and S,
        # so they are generated again before the timed one
        res["eigensolve_first_ms"], _ = timed(lambda: fl.eigensolve(H, S, vectors=vectors))
        res["generate_ms"], _ = timed(lambda: fl.hs_generate(cell, cell.kpts, g, prec=prec, out=[(H, S)]))
        res["eigensolve_ms"], out = timed(lambda: fl.eigensolve(H, S, vectors=vectors))
        w = out[0].cpu().numpy()
        res.update({"eps_min": float(w[0]), "eps_max": float(w[-1])})
    print(f"# eigen {json.dumps(res)}", flush=True)
    return res


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed graph replays of the headline path")
    ap.add_argument("--warmup", type=int, default=3, help="untimed graph replays before them")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precs", default="i8mod,fp64",
                    help="paths to measure; the first is the headline (value, roofline); others: i8, bf16 and "
                         "'+leg' variants (S through the addition theorem)")
    ap.add_argument("--slices", type=int, default=0)
    ap.add_argument("--s-method", default="gemm", choices=["gemm", "legendre"],
                    help="S method of paths without a '+leg' suffix")
    ap.add_argument("--nk", type=int, default=0, help="use only the first nk k-points (0 = all)")
    ap.add_argument("--lnonsph", type=int, default=-1,
                    help="structured T: non-spherical terms only for l', l <= lnonsph (-1: dense T, the default)")
    ap.add_argument("--eager", action="store_true",
                    help="time the headline by eager flapw_hs_generate calls instead of graph replays")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock guard: paths after the headline drop timed steps (and the radial leg is "
                         "skipped) when the run would otherwise pass this many seconds; the line records it")
    ap.add_argument("--mfma-ceiling", action="store_true",
                    help="only run the matrix-core rate microbenchmark (constant and random operands) and exit")
    ap.add_argument("--ceiling", action="store_true",
                    help="also run the matrix-core rate microbenchmark and report the headline against it")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner and use the library's default digit or modulus count and tile "
                         "band (by default each split path is tuned on k-point 0 before timing)")
    ap.add_argument("--cpu-sample", type=int, default=768,
                    help="basis functions of k-point 0 in the oracle's random principal submatrix")
    ap.add_argument("--radial-nr", type=int, default=1001,
                    help="mesh points of the radial-setup leg (radial functions and integrals of the "
                         "workload's atom types); 0 skips the leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eigen", action="store_true",
                    help="only time the generation with the interstitial terms and the generalized eigensolve "
                         "H c = eps S c of k-point 0 of --config (precision: the first of --precs) and exit")
    ap.add_argument("--oracle-times", action="store_true",
                    help="only time the CPU oracle per k-point on the named workloads 0-4 (whole k-points where "
                         "that takes minutes at most, else extrapolated from a sample; one core on the smallest) "
                         "and exit")
    ap.add_argument("--operand-study", action="store_true",
                    help="only time the modular contraction of one k-point-sized problem on random and on constant "
                         "operands (same instructions, different switching activity) and exit")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (calibrates the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters against known bytes) and exit")
    return ap


def main():
    args = make_parser().parse_args()
    t_start = time.perf_counter()

    if args.mfma_ceiling:
        print(json.dumps(mfma_ceiling()))
        return
    if args.operand_study:
        print(json.dumps(operand_study(args.config, args.slices or 11)))
        return
    if args.oracle_times:
        print(json.dumps(oracle_times(range(5))))
        return
    if args.eigen:
        print(json.dumps(eigen_leg(args.config, args.precs.split(",")[0].partition("+")[0])))
        return
    if args.copy_calib:
        import torch
        n = args.copy_calib * (1 << 20)
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": n, "copy_calib_bytes_written": n, "launches": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(k-points, being independent, would be divided among GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthcells
    from paper_1602_06589_amd import Flapw
    from paper_1602_06589_amd.flapw import FlapwError

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    cell = synthcells.config(args.config, n_k=(args.nk or None))
    nk = cell.n_k
    gdev = [torch.as_tensor(np.ascontiguousarray(g), device="cuda") for g in cell.gvecs]
    f_alg = [cell.flops_per_k(i) for i in range(nk)]
    kr = cell.k_rows()
    # algorithmic flops of the contraction kernel: S and H triangles, or H alone when S comes from
    # the addition theorem, over the rows it contracts (with S by the addition theorem and a
    # structured T, only the rows of l <= l_nonsph)
    per_mat = [8.0 * kr * cell.n_g(i) * (cell.n_g(i) + 1.0) for i in range(nk)]
    k_cut = contraction_rows(cell.lmax[cell.atom_type], args.lnonsph)
    per_mat_cut = [8.0 * k_cut * cell.n_g(i) * (cell.n_g(i) + 1.0) for i in range(nk)]
    idx = sample_indices(cell.n_g(0), args.cpu_sample)

    def split_path(path):
        prec, _, suffix = path.partition("+")
        return prec, ("legendre" if suffix == "leg" else args.s_method)
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    stream = torch.cuda.current_stream()
    print(f"# workload {cell.name}: {cell.n_atoms} atoms, {cell.n_types} types, K={kr}, {nk} k-points, "
          f"N_G {min(cell.n_g(i) for i in range(nk))}..{max(cell.n_g(i) for i in range(nk))}, "
          f"F_alg {sum(f_alg):.3e}", flush=True)

    results, samples = {}, {}
    for pi, path in enumerate(precs):
        is_head = pi == 0
        prec, s_method = split_path(path)
        f_contract = [2.0 * x for x in per_mat] if s_method == "gemm" else per_mat_cut
        n_warm, n_time, n_eager = step_plan(is_head, args.steps, args.warmup)
        use_graph = not (is_head and args.eager)
        notes = []
        with Flapw() as fl:                   # one handle per path: its work buffers are freed after
            fl.set_s_method(s_method)
            fl.set_lnonsph(args.lnonsph)
            tuned = None
            if not args.no_tune and prec != "fp64" and not args.slices:
                t0 = time.perf_counter()
                try:
                    tuned = fl.tune(cell, cell.kpts[0], gdev[0], prec=prec, tol=1e-10)
                except FlapwError as err:         # no candidate count meets the tolerance
                    tuned = {"error": str(err)}
                tuned["seconds"] = time.perf_counter() - t0
                print(f"# {path}: tuned {json.dumps(tuned)}", flush=True)
                fl.release_workspace()            # the plan below owns its own buffers
            out = [(torch.zeros((cell.n_g(i), cell.n_g(i)), dtype=torch.complex128, device="cuda"),
                    torch.zeros((cell.n_g(i), cell.n_g(i)), dtype=torch.complex128, device="cuda")) for i in range(nk)]

            def timed(run, n_w, n_t, label, guard=False):
                """n_w untimed runs, then n_t runs each between HIP events on the stream; the whole
                timed region is bracketed by synchronisations.  With guard, n_t shrinks so that the
                run keeps to the wall-clock budget (judged from the first untimed run).  Returns the
                per-run ms and the wall time."""
                t_one = None
                for w in range(n_w):
                    t0 = time.perf_counter()
                    run()
                    torch.cuda.synchronize()
                    if w == 0:
                        t_one = time.perf_counter() - t0
                torch.cuda.synchronize()
                if guard and t_one is not None:
                    left = args.budget_s - (time.perf_counter() - t_start) - 2.0 * t_one   # the eager steps
                    fit = int(left / t_one)
                    if fit < n_t:
                        n_t = max(1, fit)
                        notes.append(f"wall-clock guard: {n_t} timed run(s) of {label} "
                                     f"({max(left, 0):.0f} s left of {args.budget_s:.0f})")
                evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(n_t)]
                t0 = time.perf_counter()
                for a, b in evs:
                    a.record(stream)
                    run()
                    b.record(stream)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                per = [a.elapsed_time(b) for a, b in evs]
                print(f"# {path}: {label} {n_t} runs, median {np.median(per):.2f} ms, wall {wall:.1f} s", flush=True)
                return per, wall

            if not is_head:
                n_warm = max(1, n_warm)          # the guard judges a path by its first untimed run
            rec = {"s_method": s_method, "tuned": tuned}
            if use_graph:
                with fl.plan(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out) as plan:
                    per, wall = timed(lambda: plan.launch(stream), n_warm, n_time, "graph replay", not is_head)
                rec["timing"] = "median of HIP-graph replays (flapw_plan_launch)"
            else:
                per, wall = timed(lambda: fl.hs_generate(cell, cell.kpts, gdev, prec=prec, slices=args.slices,
                                                         out=out), n_warm, n_time, "eager", not is_head)
                rec["timing"] = "median of eager flapw_hs_generate calls"
            med = float(np.median(per))
            rec.update({"steps": n_time, "warmup": n_warm, "ms_per_step": med,
                        "ms_per_step_mean": float(np.mean(per)), "ms_per_step_min": float(np.min(per)),
                        "wall_ms_per_step": wall * 1e3 / n_time, "ms_per_kpoint": med / nk,
                        "tflops": sum(f_alg) / (med * 1e-3) / 1e12})
            # eager steps with the library's per-kernel HIP events: the stage breakdown and the
            # contraction kernel's average launch time
            if is_head:          # eager warm-up (the kernels' own event times need none)
                fl.hs_generate(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out)
            torch.cuda.synchronize()
            fl.profile(True)
            per_e, _ = timed(lambda: fl.hs_generate(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out),
                             0, n_eager, "eager (profiled)")
            kern = {fam: fl.kernel_time(fam)
                    for fam in ("coeffs", "tmat", "qpanel", "hs_fp64", "slice", "hs_split", "hs_mod", "mod_crt",
                                "leg_prep", "s_legendre")}
            fl.profile(False)
            n_l, k_ms = kern[KERNEL[prec]]
            rec.update({
                "eager_steps": n_eager, "eager_ms_per_step": float(np.mean(per_e)),
                "kernels_ms_per_step": {k: v[1] / n_eager for k, v in kern.items() if v[0]},
                "launches_per_step": {k: v[0] // n_eager for k, v in kern.items() if v[0]},
                "contraction_tflops": sum(f_contract) * n_eager / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None,
            })
            if notes:
                rec["notes"] = notes
            results[path] = rec
            print(f"# {path}: {med:.2f} ms/step, {rec['tflops']:.2f} TFLOP/s, kernels "
                  f"{json.dumps(rec['kernels_ms_per_step'])}", flush=True)
            samples[path] = (gather_block(out[0][0], idx), gather_block(out[0][1], idx))
            del out

    base = None
    if not args.no_cpu_baseline:
        base, (Ho, So) = cpu_baseline_leg(cell, idx, args.lnonsph)
        ref = {"H": np.triu(Ho), "S": np.triu(So)}
        for p in precs:
            Hs, Ss = samples[p]
            est = {"H": error_estimates(Hs, ref["H"], cell.n_g(0)), "S": error_estimates(Ss, ref["S"], cell.n_g(0))}
            results[p]["rel_err"] = {m: est[m]["full_relF_est"] for m in ("H", "S")}
            results[p]["errors"] = est
        print(f"# cpu baseline: {json.dumps(base)}", flush=True)

    radial = None
    if args.radial_nr:
        if time.perf_counter() - t_start < args.budget_s:
            radial = radial_leg(cell, args.radial_nr, 3, not args.no_cpu_baseline)
        else:
            radial = {"skipped": "wall-clock guard"}

    head_path = precs[0]
    head, head_method = split_path(head_path)
    r = results[head_path]
    n_launch = max(1, r["launches_per_step"].get(KERNEL[head], 1))
    k_ms = r["kernels_ms_per_step"].get(KERNEL[head], 0.0) / n_launch
    achieved = r["contraction_tflops"]
    # the committed counters cover the default method (S with H on the matrix cores)
    slices = args.slices or ((r["tuned"] or {}).get("slices") or DEFAULT_SLICES.get(head, 0))
    traffic = read_traffic(head, cell.name, slices) if head_method == "gemm" else None
    roof = {"bound": "mfma", "kernel": KERNEL[head], "achieved": achieved, "peak": PEAKS[head],
            # achieved counts algorithmic FP64-equivalent flops; peak is the path's own matrix-core
            # peak (int8 operations for the split paths, 5.0 POP/s = 5000 T per second)
            "unit": "TFLOP/s", "peak_unit": "TFLOP/s" if head == "fp64" else "TOP/s (int8 operations)",
            "frac": (achieved / PEAKS[head]) if achieved else None, "traffic": traffic,
            "avg_launch_ms": k_ms, "launches_per_step": n_launch,
            "flops_per_launch": (2.0 * sum(per_mat) if head_method == "gemm" else sum(per_mat_cut)) / n_launch,
            "algorithmic_unit": ("FP64-equivalent flops of the S and H upper triangles (8 K N(N+1) each)"
                                 if head_method == "gemm" else
                                 "FP64-equivalent flops of the H upper triangle (8 K' N(N+1), K' the rows the "
                                 "structured T contracts, K without one); S by the addition theorem")}
    if head != "fp64" and achieved:
        # the split path's FP64-equivalent rate against the FP64 matrix-core roofline it replaces
        roof["fp64_roofline_frac"] = achieved / PEAKS["fp64"]
        ex = achieved * executed_per_flop(slices, head)
        roof.update({"executed_ops_per_flop": executed_per_flop(slices, head), "executed_achieved": ex,
                     "executed_frac": ex / PEAKS[head], "slices": slices})
        if head == "i8mod":
            roof["bound_evidence"] = (
                "board power: on streamed random residues the int8 matrix cores issue at about 0.87 G "
                "busy cycles per second per SIMD (about 1.8 POP/s executed) for 256 x 128 and 256 x 256 "
                "blocks alike; with zero residues the same kernel runs at the full clock "
                "(profiles/power_bound_hs_mod_c4_scale.md)")
    ceil = mfma_ceiling() if args.ceiling else None
    copies = copy_ceiling() if args.ceiling and head == "i8mod" else None
    if copies:
        kp2 = -(-2 * cell.k_rows() // 256) * 256          # contraction rows, padded like the library's
        cb = [mod_copy_bytes(cell.n_g(i), kp2, slices) for i in range(len(cell.kpts))]
        rate = float(np.mean(cb)) / (roof["avg_launch_ms"] * 1e-3) / 1e12
        roof["stage_copies"] = {
            "bytes_per_launch": float(np.mean(cb)), "TBps": rate, "l2_lds_ceiling_TBps": copies["l2_lds_dma_tbs"],
            "frac": rate / copies["l2_lds_dma_tbs"], "rates": copies,
            "note": "L2 -> LDS bytes of the contraction's stage copies against the LDS-DMA rate from L2 of a "
                    "copy-only loop with the same stage structure"}
    if ceil:
        key = {"i8": "i8_random_TOPs", "i8mod": "i8_random_TOPs", "bf16": "bf16_random_TFLOPs",
               "fp64": "f64_random_TFLOPs"}[head]
        ref_rate = roof.get("executed_achieved", achieved)
        roof["ceiling_random_operands"] = {
            "rates": ceil, "value": ceil[key],
            "frac": (ref_rate / ceil[key]) if ref_rate else None,
            "note": "matrix-core rate of a register-only loop on operands distributed like this path's; "
                    "context beside the published peak, which stays the roofline"}
    fp64_key = next((p for p in precs if split_path(p) == ("fp64", head_method)), None)
    line = {
        "metric": "H+S gen time/k-point & TFLOP/s: split-prec vs FP64 MFMA at ≤1e-10 rel err",
        "value": r["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": r["steps"], "warmup": r["warmup"],
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "bf16": "bf16", "i8": "i8", "i8mod": "i8"}[head], "data": "synthetic",
        "speedup_vs_fp64": (results[fp64_key]["ms_per_step"] / r["ms_per_step"])
        if fp64_key and fp64_key != head_path else None,
        "config": {"workload": cell.name, "n_atoms": cell.n_atoms, "n_types": cell.n_types, "K": kr,
                   "lmax": int(cell.lmax.max()), "lpot": cell.lpot, "n_kpoints": nk,
                   "n_g": [cell.n_g(i) for i in range(nk)], "path": head, "slices": slices,
                   "s_method": head_method, "lnonsph": args.lnonsph},
        "ms_per_kpoint": r["ms_per_kpoint"],
        "rel_err": r.get("rel_err"),
        "roofline": roof,
        "cpu_baseline": base,
        "paths": results,
        "radial_setup": radial,
        "wall_s": time.perf_counter() - t_start,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
