#!/usr/bin/env python3
"""Benchmark: H and S generation (coefficients -> T -> per-atom panels -> S/H contractions) on
one MI355X, for the seeded synthetic workloads of synthcells.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--precs i8mod,i8,fp64,i8mod+leg,fp64+leg]
                    [--slices s | --no-tune]

A path is a precision (i8mod, i8, bf16 or fp64 for the S/H contraction) with an optional "+leg": S then
comes from the addition theorem (section 3.1) and the contraction computes H alone.  The first
path is the headline.
Before its timing, each split path runs the library's autotuner on k-point 0 (flapw_tune: the
smallest digit or modulus count whose H and S errors on a sampled block are at most 1e-10 / 4,
then the fastest tile band); --slices fixes the count instead and --no-tune takes the defaults.
A step is one flapw_hs_generate call over every k-point of the workload (the whole path).
Inputs (G lists) are resident in HBM before timing starts; K timed steps are bracketed by
torch.cuda.synchronize().  Prints one JSON line:
  value      algorithmic TFLOP/s of the headline path (the first of --precs), F_alg per k-point
             = 16 K N(N+1) + 32 N sum_a NL_a^2 (S and H upper triangles + panels T_a P_a)
  roofline   the dominant kernel (the S/H contraction), its average launch time from HIP events
             recorded by the library on the launch stream
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload; the sampled
             entries also give the relative Frobenius error of every measured path
  radial_setup  the step upstream of the coefficients and T: radial functions and the integral
             tables of the workload's atom types from synthetic radial meshes (--radial-nr points),
             GPU time per call and, beside it, the oracle's time and deviation
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
# multiply-add in the FP64 count; the modular path runs one product per modulus
def executed_per_flop(slices: int, prec: str = "i8") -> float:
    return float(slices) if prec == "i8mod" else slices * (slices + 1) / 2.0
KERNEL = {"fp64": "hs_fp64", "bf16": "hs_split", "i8": "hs_split", "i8mod": "hs_mod"}
DEFAULT_SLICES = {"i8": 6, "bf16": 6, "i8mod": 11}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def kernel_sources_sha(prec: str) -> str:
    names = {"fp64": ["contract_fp64.hip"], "i8": ["split.hip"], "bf16": ["split_bf16.hip"],
             "i8mod": ["split_mod.hip"]}[prec]
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1602_06589_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(prec: str, workload: str):
    """HBM bytes per launch of the contraction kernel from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha = kernel_sources_sha(prec)
    for line in open(TRAFFIC_FILE):
        if not line.startswith("traffic "):
            continue
        kv = dict(x.split("=", 1) for x in line.split()[1:])
        if kv.get("kernel") == KERNEL[prec] and kv.get("workload") == workload and kv.get("src_sha") == sha:
            return float(kv["bytes_per_launch"])
    return None


def cpu_baseline_leg(cell, outs, nsamp: int, lnonsph: int = -1):
    """The oracle on a bounded sample (k-point 0: an nsamp x nsamp block of basis functions,
    H and S), timed on the host cores.  Also returns the relative Frobenius error of each GPU
    path on those entries (upper triangle)."""
    import oracle
    oracle._load()
    ik = 0
    n = cell.n_g(ik)
    rng = np.random.default_rng(4242)
    idx = np.sort(rng.choice(n, min(nsamp, n), replace=False))
    t0 = time.perf_counter()
    T = oracle.tmat_all(cell, lnonsph=lnonsph)
    Ho, So = oracle.hs_sampled(cell, ik, idx, idx, T)
    dt = time.perf_counter() - t0
    k = cell.k_rows()
    nl = cell.nl_atom().astype(float)
    flops = 2 * len(idx) * len(idx) * 16.0 * k + 2 * len(idx) * 32.0 * float((nl * nl).sum())
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    up = idx[:, None] <= idx[None, :]
    errs = {}
    for prec, (H, S) in outs.items():
        Hn, Sn = H.cpu().numpy(), S.cpu().numpy()
        e = {}
        for name, M, R in (("H", Hn, Ho), ("S", Sn, So)):
            got = M[np.ix_(idx, idx)].T
            e[name] = float(np.linalg.norm((got - R)[up]) / np.linalg.norm(R[up]))
        errs[prec] = e
    base = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"k-point 0 of {cell.name}: H and S on a {len(idx)}x{len(idx)} block of basis functions "
                      f"(coefficients of those columns, T, per-atom panels), {dt:.1f} s",
            "seconds": dt}
    return base, errs


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precs", default="i8mod,i8,fp64,i8mod+leg,fp64+leg",
                    help="paths to measure; the first is the headline (value, roofline)")
    ap.add_argument("--slices", type=int, default=0)
    ap.add_argument("--s-method", default="gemm", choices=["gemm", "legendre"],
                    help="S method of paths without a '+leg' suffix")
    ap.add_argument("--nk", type=int, default=0, help="use only the first nk k-points (0 = all)")
    ap.add_argument("--lnonsph", type=int, default=-1,
                    help="structured T: non-spherical terms only for l', l <= lnonsph (-1: dense T, the default)")
    ap.add_argument("--mfma-ceiling", action="store_true",
                    help="only run the matrix-core rate microbenchmark (constant and random operands) and exit")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the matrix-core rate microbenchmark")
    ap.add_argument("--graph", action="store_true",
                    help="also time replays of the generation captured in a HIP graph (flapw_plan_*)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner and use the library's default digit or modulus count and tile "
                         "band (by default each split path is tuned on k-point 0 before timing: the smallest "
                         "count whose sampled error is at most 1e-10 / 4, then the fastest band)")
    ap.add_argument("--cpu-sample", type=int, default=384)
    ap.add_argument("--radial-nr", type=int, default=1001,
                    help="mesh points of the radial-setup leg (radial functions and integrals of the "
                         "workload's atom types); 0 skips the leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (calibrates the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters against known bytes) and exit")
    args = ap.parse_args()

    if args.mfma_ceiling:
        print(json.dumps(mfma_ceiling()))
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
    # the addition theorem
    per_mat = [8.0 * kr * cell.n_g(i) * (cell.n_g(i) + 1.0) for i in range(nk)]

    def split_path(path):
        prec, _, suffix = path.partition("+")
        return prec, ("legendre" if suffix == "leg" else args.s_method)
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    stream = torch.cuda.current_stream()
    print(f"# workload {cell.name}: {cell.n_atoms} atoms, {cell.n_types} types, K={kr}, {nk} k-points, "
          f"N_G {min(cell.n_g(i) for i in range(nk))}..{max(cell.n_g(i) for i in range(nk))}, "
          f"F_alg {sum(f_alg):.3e}", flush=True)

    results, outs = {}, {}
    for path in precs:
        prec, s_method = split_path(path)
        f_contract = [(2.0 if s_method == "gemm" else 1.0) * x for x in per_mat]
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
            out = [(torch.zeros((cell.n_g(i), cell.n_g(i)), dtype=torch.complex128, device="cuda"),
                    torch.zeros((cell.n_g(i), cell.n_g(i)), dtype=torch.complex128, device="cuda")) for i in range(nk)]
            for _ in range(args.warmup):
                fl.hs_generate(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out)
            torch.cuda.synchronize()
            fl.profile(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            for _ in range(args.steps):
                fl.hs_generate(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms = e0.elapsed_time(e1) / args.steps
            kern = {fam: fl.kernel_time(fam)
                    for fam in ("coeffs", "tmat", "qpanel", "hs_fp64", "slice", "hs_split", "hs_mod", "mod_crt",
                                "leg_prep", "s_legendre")}
            fl.profile(False)
            n_l, k_ms = kern[KERNEL[prec]]
            achieved = sum(f_contract) * args.steps / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None
            results[path] = {
                "s_method": s_method, "tuned": tuned, "ms_per_step": ms, "wall_s": wall, "ms_per_kpoint": ms / nk,
                "tflops": sum(f_alg) / (ms * 1e-3) / 1e12,
                "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kern.items() if v[0]},
                "launches_per_step": {k: v[0] // args.steps for k, v in kern.items() if v[0]},
                "contraction_tflops": achieved,
            }
            print(f"# {path}: {ms:.2f} ms/step, {results[path]['tflops']:.2f} TFLOP/s, kernels "
                  f"{json.dumps(results[path]['kernels_ms_per_step'])}", flush=True)
            if args.graph:
                with fl.plan(cell, cell.kpts, gdev, prec=prec, slices=args.slices, out=out) as plan:
                    plan.launch()
                    torch.cuda.synchronize()
                    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    g0.record(stream)
                    for _ in range(args.steps):
                        plan.launch(stream)
                    g1.record(stream)
                    torch.cuda.synchronize()
                    results[path]["graph_ms_per_step"] = g0.elapsed_time(g1) / args.steps
                print(f"# {path}: graph replay {results[path]['graph_ms_per_step']:.2f} ms/step", flush=True)
            outs[path] = (out[0][0], out[0][1])       # k-point 0 is what the CPU baseline samples
            del out

    base, errs = (None, {})
    if not args.no_cpu_baseline:
        base, errs = cpu_baseline_leg(cell, outs, args.cpu_sample, args.lnonsph)
        for p in precs:
            results[p]["rel_err"] = errs[p]

    radial = radial_leg(cell, args.radial_nr, args.steps, not args.no_cpu_baseline) if args.radial_nr else None

    head_path = precs[0]
    head, head_method = split_path(head_path)
    r = results[head_path]
    n_launch = max(1, r["launches_per_step"].get(KERNEL[head], 1))
    k_ms = r["kernels_ms_per_step"].get(KERNEL[head], 0.0) / n_launch
    achieved = r["contraction_tflops"]
    # the committed counters cover the default method (S with H on the matrix cores)
    traffic = read_traffic(head, cell.name) if head_method == "gemm" else None
    slices = args.slices or ((r["tuned"] or {}).get("slices") or DEFAULT_SLICES.get(head, 0))
    roof = {"bound": "mfma", "kernel": KERNEL[head], "achieved": achieved, "peak": PEAKS[head],
            "unit": "TFLOP/s" if head == "fp64" else "TOP/s",
            "frac": (achieved / PEAKS[head]) if achieved else None, "traffic": traffic,
            "avg_launch_ms": k_ms, "launches_per_step": n_launch,
            "flops_per_launch": sum(per_mat) * (2.0 if head_method == "gemm" else 1.0) / n_launch,
            "algorithmic_unit": ("FP64-equivalent flops of the S and H upper triangles (8 K N(N+1) each)"
                                 if head_method == "gemm" else
                                 "FP64-equivalent flops of the H upper triangle (8 K N(N+1)); S by the addition theorem")}
    if head != "fp64" and achieved:
        # the split path's FP64-equivalent rate against the FP64 matrix-core roofline it replaces
        roof["fp64_roofline_frac"] = achieved / PEAKS["fp64"]
        ex = achieved * executed_per_flop(slices, head)
        roof.update({"executed_ops_per_flop": executed_per_flop(slices, head), "executed_achieved": ex,
                     "executed_frac": ex / PEAKS[head], "slices": slices})
    ceil = None if args.no_ceiling else mfma_ceiling()
    if ceil:
        key = {"i8": "i8_random_TOPs", "i8mod": "i8_random_TOPs", "bf16": "bf16_random_TFLOPs",
               "fp64": "f64_random_TFLOPs"}[head]
        ref = roof.get("executed_achieved", achieved)
        roof["ceiling_random_operands"] = {
            "rates": ceil, "value": ceil[key],
            "frac": (ref / ceil[key]) if ref else None,
            "note": "matrix-core rate of a register-only loop on operands distributed like this path's "
                    "(power-limited clock); context beside the published peak, which stays the roofline"}
    line = {
        "metric": "H+S gen time/k-point & TFLOP/s: split-prec vs FP64 MFMA at ≤1e-10 rel err",
        "value": r["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "bf16": "bf16", "i8": "i8", "i8mod": "i8"}[head], "data": "synthetic",
        "speedup_vs_fp64": (results["fp64"]["ms_per_step"] / r["ms_per_step"]) if "fp64" in results and head_path != "fp64" else None,
        "config": {"workload": cell.name, "n_atoms": cell.n_atoms, "n_types": cell.n_types, "K": kr,
                   "lmax": int(cell.lmax.max()), "lpot": cell.lpot, "n_kpoints": nk,
                   "n_g": [cell.n_g(i) for i in range(nk)], "path": head, "slices": args.slices,
                   "s_method": head_method, "lnonsph": args.lnonsph},
        "ms_per_kpoint": r["ms_per_kpoint"],
        "roofline": roof,
        "cpu_baseline": base,
        "paths": results,
        "radial_setup": radial,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
