#!/usr/bin/env python3
"""Benchmark of the FFT product (eq. 11) on one MI355X, with the capacitance solve times.

One step = one batched application of the operator of eq. (4) through the FFT product
to all m right-hand sides of the workload (the unit of work of every GMRES iteration),
in the precision the mixed solve uses for its inner iterations (FP32 FFT and block
multiply; FP64 input, output and diagonal term).  value = RHS-products per second.

Also reported: the FP64 product rate, the C-matrix solve time in FP64 and in mixed
precision at the same accuracy, a roofline entry for the dominant pass (algorithmic
bytes from the library's byte model / live HIP-event durations), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "plates": "two 48x48x2-voxel plates 8 voxels apart on a 64x64x32 grid, eps_r=4 gap, dv=1um, 2 RHS",
    "cube16": "unit cube on a 16^3 grid, vacuum, 1 RHS",
    "random128": "8 random conductor boxes in 6 dielectric boxes on a 128^3 grid (seed 3), 8 RHS",
    "meander": "4 meander lines (11 runs) on an eps_r=4.4 substrate, 512x512x16 grid, 4 RHS",
    "grad256": "6 conductors in a 4x4-tiled substrate (16 eps blocks), 256x256x64 grid, 6 RHS",
}


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_02609_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".h")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(config, kernel, prec):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (null when absent or
    taken on a different kernel source)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}_{prec}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("passes", {}).get(kernel)


def cpu_baseline(scene, nrhs, budget_s=20.0):
    """FP64 oracle: dense rows of eq. (4) assembled for a row sample, then the dense
    product of that row block timed and scaled to a full N-row product."""
    import numpy as np

    import oracle
    from oracle import dense
    cores = len(os.sched_getaffinity(0))
    p = oracle.panelize(scene["cond_id"], scene["eps_r"], scene["eps_b"])
    N = len(p["axis"])
    rng = np.random.default_rng(0)
    nrow = min(N, 512)
    rows = np.sort(rng.choice(N, nrow, replace=False))
    t0 = time.perf_counter()
    A = dense.assemble_rows(p, rows)
    t_asm = time.perf_counter() - t0
    X = rng.standard_normal((N, nrhs))
    reps = 0
    t0 = time.perf_counter()
    while True:
        A @ X
        reps += 1
        el = time.perf_counter() - t0
        if el > min(5.0, budget_s) or reps >= 2000:
            break
    t_block = el / reps
    t_full = t_block * N / nrow
    return {"value": nrhs / t_full, "unit": "RHS-MVPs/s", "cores": cores, "kind": "oracle",
            "sample": (f"{nrow} random rows of the dense eq.(4) matrix (N={N}) assembled by the oracle in "
                       f"{t_asm:.1f}s ({t_asm / nrow * N:.0f}s extrapolated to all rows, not counted), "
                       f"row-block product with {nrhs} RHS timed over {reps} reps and scaled by N/rows"),
            "assembly_s_per_row": t_asm / nrow}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="plates", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is design-only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2004_02609_amd import voxcap

    dev = torch.device("cuda:0")
    scene = scenes.by_name(args.config)
    t0 = time.perf_counter()
    P = voxcap.Problem.from_scene(scene).setup()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    B, N = P.m, P.N
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev).manual_seed(0)
    x = torch.randn(B, N, dtype=torch.float64, device=dev, generator=g)
    y = torch.empty_like(x)

    def run(prec, steps, warm, profile):
        for _ in range(warm):
            P.apply(x, y, prec=prec, stream=stream)
        torch.cuda.synchronize()
        P.pass_times()                       # drop anything recorded before
        P.profile(profile)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            P.apply(x, y, prec=prec, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        P.profile(False)
        ms = e0.elapsed_time(e1)
        return ms, P.pass_times()

    print(f"# {args.config}: N={N} m={B} fft={P.fft_size()} setup {t_setup:.2f}s", file=sys.stderr, flush=True)
    ms, (pms, pcnt, pbytes) = run(args.prec, args.steps, args.warmup, True)
    value = args.steps * B / (ms / 1e3)
    other = "fp64" if args.prec == "fp32" else "fp32"
    ms_o, _ = run(other, max(10, args.steps // 2), 3, False)
    value_o = max(10, args.steps // 2) * B / (ms_o / 1e3)
    print(f"# {args.prec} product {ms / args.steps * 1e3:.1f} us/step, {other} "
          f"{ms_o / max(10, args.steps // 2) * 1e3:.1f} us/step", file=sys.stderr, flush=True)

    dom = int(np.argmax(pms))
    avg_ms = pms[dom] / max(1, pcnt[dom])
    achieved = pbytes[dom] / (avg_ms / 1e3) / 1e9
    kname = voxcap.PASS_NAMES[dom]
    traffic = load_traffic(args.config, kname, args.prec)
    passes = {voxcap.PASS_NAMES[i]: {"avg_us": pms[i] / max(1, pcnt[i]) * 1e3, "launches": pcnt[i],
                                     "alg_bytes": pbytes[i],
                                     "alg_GBs": pbytes[i] / (pms[i] / max(1, pcnt[i]) / 1e3) / 1e9
                                     if pms[i] > 0 else None}
              for i in range(5)}

    solve = None
    if not args.no_solve:
        solve = {}
        Cref, st_ref = P.capacitance(prec="fp64", rtol=1e-12)
        for mode in ("fp64", "mixed"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Cm, st = P.capacitance(prec=mode, rtol=1e-9)
            t = time.perf_counter() - t0
            d = np.abs(np.diag(Cref)).max()
            gate = np.abs(Cref) >= 1e-3 * d
            err = float((np.abs(Cm - Cref)[gate] / np.abs(Cref)[gate]).max())
            solve[mode] = {"time_s": t, "iters": st["iters"], "ir_steps": st["ir_steps"],
                           "max_rel_err_vs_fp64_1e-12": err, "products": st["mvp_count"]}
        solve["speedup_mixed_vs_fp64"] = solve["fp64"]["time_s"] / solve["mixed"]["time_s"]

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(scene, B)

    line = {
        "metric": "FFT-MVPs/s + C-matrix solve time @1e-6 rel err, mixed/batched vs FP64 plain",
        "value": value, "unit": "RHS-MVPs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "panels": N, "rhs": B,
                   "fft_size": list(P.fft_size()), "product_precision": args.prec},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "other_precision": {"prec": other, "value": value_o, "unit": "RHS-MVPs/s"},
        "passes": passes,
        "solve": solve,
        "setup_s": t_setup,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
