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
# vector peaks of MI355X (256 CUs x 2.4 GHz): FP32 157.3 TFLOP/s (two FP32 FMAs per
# lane per clock), FP64 78.6 TFLOP/s
VEC_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


def xpass_flops(fft, nrhs, nout):
    """Algorithmic flops of one x-pass launch (forward x transform of the 3 input
    components, per-frequency block multiply, inverse x transform of the nout outputs)
    per (ky, kz) column and right-hand side: 5 L log2 L per length-L complex transform,
    4 flops per real-by-complex multiply-accumulate of the block product, 6 per complex
    half-voxel phase factor (one per input and output component)."""
    import math
    L, My, Mz = fft
    cols = My * (Mz // 2 + 1)
    per = (3 + nout) * 5.0 * L * math.log2(L) + L * (4.0 * 3 * nout + 6.0 * (3 + nout))
    return cols * nrhs * per
WORKLOADS = {
    "plates": "two 48x48x2-voxel plates 8 voxels apart on a 64x64x32 grid, eps_r=4 gap, dv=1um, 2 RHS",
    "cube16": "unit cube on a 16^3 grid, vacuum, 1 RHS",
    "random128": "8 random conductor boxes in 6 dielectric boxes on a 128^3 grid (seed 3), 8 RHS",
    "meander": "4 meander lines (11 runs) on an eps_r=4.4 substrate, 512x512x16 grid, 4 RHS",
    "grad256": "6 conductors in a 4x4-tiled substrate (16 eps blocks), 256x256x64 grid, 6 RHS",
}


# sources of the product's pass kernels (device code and the launch structs they take):
# a traffic summary is only reported while these are what it was measured on
PRODUCT_KERNEL_SOURCES = ["fft_core.hpp", "mvp_kernels.h", "mvp_kernels.hip", "sandwich_impl.hpp", "ypass_impl.hpp",
                          "sandwich_f32_33.hip", "sandwich_f32_36.hip", "sandwich_f32_63.hip", "sandwich_f64_33.hip",
                          "sandwich_f64_36.hip", "sandwich_f64_63.hip", "ypass_f32.hip", "ypass_f64.hip"]


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_02609_amd", "csrc")
    for f in PRODUCT_KERNEL_SOURCES:
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


def _pmc_rows(d, counter):
    """(dispatch id, kernel name, value) of one counter from a rocprofv3 --pmc csv run."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            name = r.get("Kernel_Name", "")
            rows[k] = (name, rows.get(k, (name, 0.0))[1] + float(r["Counter_Value"]))
    return [(k, v[0], v[1]) for k, v in sorted(rows.items())]


def write_traffic(args):
    """HBM bytes per launch of each pass of the timed steps: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) scaled so the calibration copy reads and writes its known size."""
    fetch = _pmc_rows(args.write_traffic[0], "FETCH_SIZE")
    write = _pmc_rows(args.write_traffic[1], "WRITE_SIZE")
    copy_bytes = float(args.calib_copy_mib) * (1 << 20)
    if copy_bytes <= 0:
        raise SystemExit("--write-traffic needs the --calib-copy-mib of the profiled runs")
    tname = "float" if args.prec == "fp32" else "double"
    # the y pass runs on one of two kernels (the autotuner's choice): the timed steps'
    # y launches are the last 2 x steps of either, alternating forward / inverse
    kern = {"zfwd_scatter": ("k_zfwd<" + tname,), "y": ("k_strided<" + tname, "k_ypass<" + tname),
            "x_sandwich_multiply": ("k_xsandwich<" + tname,), "zinv_gather": ("k_zinv<" + tname,)}

    def per_pass(rows):
        cp = [v for _, n, v in rows if "copy" in n.lower()]
        if not cp:
            raise SystemExit("calibration copy kernel not found")
        scale = copy_bytes / (max(cp) * 1024.0)
        out = {}
        for p, key in kern.items():
            vals = [v for _, n, v in rows if any(k in n.replace(" ", "") for k in key)]
            if p == "y":
                last = vals[-2 * args.steps:]
                out["y_forward"] = sum(last[0::2]) / args.steps * 1024.0 * scale
                out["y_inverse"] = sum(last[1::2]) / args.steps * 1024.0 * scale
            else:
                last = vals[-args.steps:]
                out[p] = sum(last) / len(last) * 1024.0 * scale
        return out, scale, max(cp)

    f, fs, fcp = per_pass(fetch)
    w, ws, wcp = per_pass(write)
    cmd = (f"python bench.py --config {args.config} --prec {args.prec} --steps {args.steps} --warmup {args.warmup} "
           f"--no-cpu --no-solve --no-other --tucker-tol 0 --toeplitz-tol 0 --batch 0 --calib-copy-mib {args.calib_copy_mib}")
    res = {"source_hash": kernel_source_hash(), "config": args.config, "prec": args.prec,
           "commands": [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- {cmd}",
                        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- {cmd}"],
           "copy_bytes": copy_bytes, "copy_fetch_kib": fcp, "copy_write_kib": wcp,
           "scale_fetch": fs, "scale_write": ws,
           "passes": {p: f[p] + w[p] for p in f},
           "fetch_bytes": f, "write_bytes": w}
    path = os.path.join(ROOT, "profiles", f"traffic_{args.config}_{args.prec}.json")
    with open(path, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


def tucker_run(args, scene, x, stream, B, ms_product_full):
    """The same product with the spectra Tucker-compressed (eq. 13) and rebuilt on the
    matrix cores before each product: compression ratio, rebuild time, the paper's
    computational overhead CO = rebuild time / one product, and the rebuild's MFMA
    rate (dense GEMM flops of the three mode products) and output bandwidth."""
    import torch

    from paper_2004_02609_amd import voxcap
    Pt = voxcap.Problem.from_scene(scene).setup(tucker_tol=args.tucker_tol, autotune=not args.no_tune,
                                                precisions=2 if args.prec == "fp32" else 1)
    y = torch.empty_like(x)
    for _ in range(3):
        Pt.apply(x, y, prec=args.prec, stream=stream)
    torch.cuda.synchronize()
    Pt.tucker_info()                       # drop what was recorded before
    base = Pt.tucker_info()
    steps = max(5, args.steps // 4)
    # product rate without timing events, then the rebuild's own time with events
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        Pt.apply(x, y, prec=args.prec, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    Pt.profile(1)
    for _ in range(steps):
        Pt.apply(x, y, prec=args.prec, stream=stream)
    torch.cuda.synchronize()
    Pt.profile(0)
    Pt.pass_times()
    info = Pt.tucker_info()
    n_rb = info["rebuilds"] - base["rebuilds"]
    rb_ms = (info["rebuild_ms"] - base["rebuild_ms"]) / max(1, n_rb)
    D = (Pt.fft_size()[0] // 2 + 1, Pt.fft_size()[1] // 2 + 1, Pt.fft_size()[2] // 2 + 1)
    flops = 0.0
    out_bytes = 0.0
    elem = 4 if args.prec == "fp32" else 8
    for r1, r2, r3 in info["ranks"]:
        flops += 2.0 * (r1 * r2 * r3 * D[2] + r1 * r2 * D[1] * D[2] + r1 * D[0] * D[1] * D[2])
        out_bytes += elem * (D[0] * D[1] * D[2] + 2 * r1 * D[1] * D[2])   # X written, T2 written and read
    tf = flops / (rb_ms / 1e3) / 1e12
    return {"tol": args.tucker_tol, "ranks": info["ranks"], "compression_ratio": info["compression_ratio"],
            "product_ms_with_rebuild": ms, "rebuild_ms": rb_ms,
            "computational_overhead": rb_ms / ms_product_full,
            "rhs_products_per_s": B / (ms / 1e3),
            "rebuild_mfma": {"flops": flops, "achieved_tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[args.prec],
                             "frac": tf / MFMA_PEAK_TFLOPS[args.prec]},
            "rebuild_hbm": {"bytes": out_bytes, "achieved_gbs": out_bytes / (rb_ms / 1e3) / 1e9,
                            "peak_gbs": HBM_PEAK_GBS}}


def toeplitz_run(args, scene, x):
    """Toeplitz setup path (Sec. II.C, Tab. I): a cache built over a larger grid (each axis
    twice the workload's, at most 256 and at least the workload's), saved and loaded
    back, then a fresh setup of the workload from it beside a fresh direct setup."""
    import tempfile

    import numpy as np
    import torch

    from paper_2004_02609_amd import voxcap
    n = tuple(int(v) for v in scene["cond_id"].shape)
    nmax = tuple(max(a, min(2 * a, 256)) for a in n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cache = voxcap.ToeplitzCache.build(nmax, args.toeplitz_tol)
    t_build = time.perf_counter() - t0
    info = cache.info()
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "toeplitz.vct")
        t0 = time.perf_counter()
        cache.save(path)
        t_save = time.perf_counter() - t0
        file_bytes = os.path.getsize(path)
        cache.close()
        t0 = time.perf_counter()
        cache = voxcap.ToeplitzCache.load(path)
        t_load = time.perf_counter() - t0
    # restored tensors of this grid against the ones computed from the integrals
    errs = []
    for q in range(15):
        ref = voxcap.toeplitz_octant(q, n)
        errs.append(float(torch.linalg.norm(cache.restore(q, n) - ref) / torch.linalg.norm(ref)))
    Pd = voxcap.Problem.from_scene(scene)
    Pd.setup(autotune=False)
    Pc = voxcap.Problem.from_scene(scene)
    Pc.set_toeplitz_source(cache)
    Pc.setup(autotune=False)
    yd = Pd.apply(x, prec="fp64")
    yc = Pc.apply(x, prec="fp64")
    diff = float((yc - yd).abs().max() / yd.abs().max())
    td, tc = Pd.setup_time(), Pc.setup_time()
    out = {"nmax": list(nmax), "grid": list(n), "tol": args.toeplitz_tol, "build_s": t_build, "save_s": t_save,
           "load_s": t_load, "file_bytes": file_bytes, "stored_numbers": info["stored_numbers"],
           "octant_numbers": info["full_numbers"], "compression_ratio": info["compression_ratio"],
           "rank_max": int(max(max(r) for r in info["ranks"])),
           "restored_vs_computed_rel_err_max": max(errs),
           "setup_direct": {"total_s": td["total_s"], "toeplitz_s": td["toeplitz_s"]},
           "setup_from_cache": {"total_s": tc["total_s"], "toeplitz_s": tc["toeplitz_s"]},
           "toeplitz_speedup": td["toeplitz_s"] / tc["toeplitz_s"] if tc["toeplitz_s"] > 0 else None,
           "fp64_product_rel_diff_vs_direct": diff}
    del Pd, Pc
    cache.close()
    return out


def batch_run(args):
    """Uneven batch: `args.batch` independent random scenes (grid edges U{16..64}, 1-4
    conductors, half with a dielectric box) solved in mixed precision as one packed set
    (every pass of the product one launch over all scenes, each restart cycle one graph
    launch) and one after another; rtol 1e-9."""
    import numpy as np
    import torch

    import scenes
    from paper_2004_02609_amd import voxcap
    ss = scenes.uneven_batch(args.batch)
    t0 = time.perf_counter()
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    pk = voxcap.Pack(probs)
    pk.capacitance(prec="mixed", rtol=1e-9)          # captures the cycle graphs
    for P in probs:
        P.capacitance(prec="mixed", rtol=1e-9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Cb, stb = pk.capacitance(prec="mixed", rtol=1e-9)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    Cs = [P.capacitance(prec="mixed", rtol=1e-9)[0] for P in probs]
    t_seq = time.perf_counter() - t0
    diff = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(Cb, Cs))
    inf = pk.info()
    cached = None
    if args.toeplitz_tol > 0:
        # the same scenes set up from one Toeplitz cache over the batch's largest grid
        nmax = tuple(max(int(s["cond_id"].shape[a]) for s in ss) for a in range(3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cache = voxcap.ToeplitzCache.build(nmax, args.toeplitz_tol)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        probs_c = []
        for s in ss:
            Pc = voxcap.Problem.from_scene(s)
            Pc.set_toeplitz_source(cache)
            probs_c.append(Pc.setup())
        torch.cuda.synchronize()
        t_setup_c = time.perf_counter() - t0
        cache.close()
        pk_c = voxcap.Pack(probs_c)
        Cc, _ = pk_c.capacitance(prec="mixed", rtol=1e-9)
        dc = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(Cc, Cb))
        cached = {"nmax": list(nmax), "tol": args.toeplitz_tol, "cache_build_s": t_build, "setup_s": t_setup_c,
                  "setup_speedup": t_setup / t_setup_c, "max_rel_diff_C_vs_direct": dc}
        pk_c.close()
        del probs_c
    return {"scenes": len(ss), "panels_total": int(sum(P.N for P in probs)), "pack": inf,
            "setup_from_toeplitz_cache": cached,
            "ir_steps": int(stb[0]["ir_steps"]), "max_iters": int(max(max(t["iters"]) for t in stb)),
            "conductors_total": int(sum(P.m for P in probs)), "setup_s": t_setup,
            "batched_solve_s": t_batch, "sequential_solve_s": t_seq, "speedup": t_seq / t_batch,
            "scenes_per_s_batched": len(ss) / t_batch, "max_rel_diff_batch_vs_single": diff}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="plates", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="heuristic x-pass configuration instead of the autotuner")
    ap.add_argument("--no-other", action="store_true", help="skip the product in the other precision")
    ap.add_argument("--batch", type=int, default=32,
                    help="also solve this many uneven random scenes (edges 16-64) as one packed set and one by one "
                         "(0: skip)")
    ap.add_argument("--tucker-tol", type=float, default=1e-8,
                    help="also run the product with Tucker-compressed spectra at this tolerance (0: skip)")
    ap.add_argument("--toeplitz-tol", type=float, default=1e-8,
                    help="also build a Toeplitz cache over a larger grid at this tolerance and set the workload up "
                         "from it (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (HBM-counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="(no GPU) turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this command with "
                         "--calib-copy-mib into profiles/traffic_<config>_<prec>.json, then exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is design-only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2004_02609_amd import voxcap

    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    scene = scenes.by_name(args.config)
    t0 = time.perf_counter()
    P = voxcap.Problem.from_scene(scene).setup(autotune=not args.no_tune)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    B, N = P.m, P.N
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev).manual_seed(0)
    x = torch.randn(B, N, dtype=torch.float64, device=dev, generator=g)
    y = torch.empty_like(x)

    def run(prec, steps, warm, level, every=1):
        # level 2: HIP events around the x pass only (the timed run, on every `every`-th
        # step: each event adds a few us between the launches it separates); level 1:
        # around every pass (the breakdown run)
        for _ in range(warm):
            P.apply(x, y, prec=prec, stream=stream)
        torch.cuda.synchronize()
        P.pass_times()                       # drop anything recorded before
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for k in range(steps):
            P.profile(level if k % every == 0 else 0)
            P.apply(x, y, prec=prec, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        P.profile(0)
        ms = e0.elapsed_time(e1)
        return ms, P.pass_times()

    print(f"# {args.config}: N={N} m={B} fft={P.fft_size()} setup {t_setup:.2f}s", file=sys.stderr, flush=True)
    every = max(1, min(10, args.steps // 10))
    ms, (pms, pcnt, pbytes) = run(args.prec, args.steps, args.warmup, 2, every)
    value = args.steps * B / (ms / 1e3)
    # per-pass breakdown: a separate, shorter run with events around every pass
    _, (bms, bcnt, bbytes) = run(args.prec, max(10, min(args.steps, 50)), 2, 1)
    other = "fp64" if args.prec == "fp32" else "fp32"
    value_o = None
    if not args.no_other:
        ms_o, _ = run(other, max(10, args.steps // 2), 3, 0)
        value_o = max(10, args.steps // 2) * B / (ms_o / 1e3)
        print(f"# {args.prec} product {ms / args.steps * 1e3:.1f} us/step, {other} "
              f"{ms_o / max(10, args.steps // 2) * 1e3:.1f} us/step", file=sys.stderr, flush=True)

    dom = int(np.argmax(bms))
    avg_ms = bms[dom] / max(1, bcnt[dom])
    achieved = bbytes[dom] / (avg_ms / 1e3) / 1e9
    kname = voxcap.PASS_NAMES[dom]
    traffic = load_traffic(args.config, kname, args.prec)
    # the x pass does ~30 flops per algorithmic byte (nine transforms per column) and is
    # bound by vector-instruction issue, not HBM: report it against the vector peak
    nout = 6 if P.n_diel > 0 else 3
    xi = voxcap.PASS_NAMES.index("x_sandwich_multiply")
    x_ms = pms[xi] / max(1, pcnt[xi])
    x_flops = xpass_flops(P.fft_size(), B, nout)
    x_tflops = x_flops / (x_ms / 1e3) / 1e12
    x_traffic = load_traffic(args.config, "x_sandwich_multiply", args.prec)
    roofline = {"bound": "alu", "kernel": "x_sandwich_multiply", "achieved": x_tflops,
                "peak": VEC_PEAK_TFLOPS[args.prec], "unit": "TFLOP/s", "frac": x_tflops / VEC_PEAK_TFLOPS[args.prec],
                "traffic": x_traffic, "alg_flops": x_flops, "alg_bytes": pbytes[xi], "avg_us": x_ms * 1e3,
                "hbm_achieved_GBs": pbytes[xi] / (x_ms / 1e3) / 1e9,
                "hbm_frac": pbytes[xi] / (x_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                "timed_launches": pcnt[xi], "event_sampling": f"every {every}th of the {args.steps} timed steps"}
    passes = {voxcap.PASS_NAMES[i]: {"avg_us": bms[i] / max(1, bcnt[i]) * 1e3, "launches": bcnt[i],
                                     "alg_bytes": bbytes[i],
                                     "alg_GBs": bbytes[i] / (bms[i] / max(1, bcnt[i]) / 1e3) / 1e9
                                     if bms[i] > 0 else None}
              for i in range(5)}

    solve = None
    if not args.no_solve:
        solve = {}
        Cref, st_ref = P.capacitance(prec="fp64", rtol=1e-12)
        dmax = np.abs(np.diag(Cref)).max()
        gate = np.abs(Cref) >= 1e-3 * dmax

        def cerr(Cm):
            return float((np.abs(Cm - Cref)[gate] / np.abs(Cref)[gate]).max())

        def timed(mode, rtol):
            """Median of three warm solves (the restart-cycle graphs are captured by a first,
            untimed solve), with the entrywise error of the last against FP64 at 1e-12."""
            P.capacitance(prec=mode, rtol=rtol)
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Cm, st = P.capacitance(prec=mode, rtol=rtol)
                ts.append(time.perf_counter() - t0)
            return {"time_s": float(np.median(ts)), "times_s": ts, "iters": st["iters"], "ir_steps": st["ir_steps"],
                    "max_rel_err_vs_fp64_1e-12": cerr(Cm), "products": st["mvp_count"], "rtol": rtol}

        # the metric's accuracy: the loosest GMRES tolerance at which both the FP64 and the
        # mixed solve give every gated entry of C within 1e-6 of the FP64 reference
        cal = 1e-10
        for rt in (1e-5, 1e-6, 1e-7, 1e-8, 1e-9):
            if all(cerr(P.capacitance(prec=mode, rtol=rt)[0]) <= 1e-6 for mode in ("fp64", "mixed")):
                cal = rt
                break
        solve["rtol_for_1e-6"] = cal
        for mode in ("fp64", "mixed"):
            solve[mode] = timed(mode, cal)
        solve["speedup_mixed_vs_fp64"] = solve["fp64"]["time_s"] / solve["mixed"]["time_s"]
        # the same pair at a fixed, tighter tolerance
        solve["at_rtol_1e-9"] = {mode: timed(mode, 1e-9) for mode in ("fp64", "mixed")}
        solve["at_rtol_1e-9"]["speedup_mixed_vs_fp64"] = (solve["at_rtol_1e-9"]["fp64"]["time_s"] /
                                                          solve["at_rtol_1e-9"]["mixed"]["time_s"])
        # the FP64 solve with the restart cycle's kernels issued one by one
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.capacitance(prec="fp64", rtol=cal, graph=False)
        solve["fp64_no_graph_time_s"] = time.perf_counter() - t0

    tucker = None
    if args.tucker_tol > 0:
        tucker = tucker_run(args, scene, x, stream, B, ms / args.steps)

    toeplitz = None
    if args.toeplitz_tol > 0:
        toeplitz = toeplitz_run(args, scene, x)

    batch = None
    if args.batch > 0:
        batch = batch_run(args)

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
        "roofline": roofline,
        "product_hbm": {"dominant_pass": kname, "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS,
                        "traffic": traffic,
                        "all_passes_alg_bytes": float(sum(bbytes)),
                        "all_passes_GBs": float(sum(bbytes)) / (ms / args.steps / 1e3) / 1e9},
        "cpu_baseline": cpu,
        "other_precision": {"prec": other, "value": value_o, "unit": "RHS-MVPs/s"} if value_o else None,
        "passes": passes,
        "solve": solve,
        "setup_s": t_setup,
        "xpass_tuning": P.tuning_report().strip().splitlines(),
        "tucker": tucker,
        "toeplitz_setup": toeplitz,
        "batch": batch,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
