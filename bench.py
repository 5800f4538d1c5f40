#!/usr/bin/env python3
"""Benchmark of the FFT product (eq. 11) on one MI355X, with the capacitance solve times.

One step = one batched application of the operator of eq. (4) through the FFT product
to all m right-hand sides of the workload (the unit of work of every GMRES iteration),
in the form the workload's mixed solve uses for its inner iterations: FP32 FFT and
block multiply (FP64 input, output and diagonal term), and for the meander lines
(the default) the kernel spectra Tucker-compressed at 1e-8 and rebuilt on the matrix
cores inside every step (eq. 13).  value = RHS-products per second.

Also reported: the uncompressed FP32 and the FP64-plain product rates, the C-matrix
solve time in mixed precision (the step's form) and in FP64 plain at the same accuracy,
a roofline entry for the dominant pass (live HIP-event durations), and the FP64 CPU
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


def load_traffic(config, kernel, prec, tucker_tol=0.0):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (null when absent,
    taken on a different kernel source, or on the other form of the spectra: stored, or
    Tucker-compressed and built in the x pass)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}_{prec}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_hash") != kernel_source_hash():
        return None
    if (float(t.get("tucker_tol", 0.0)) > 0) != (tucker_tol > 0):
        return None
    return t.get("passes", {}).get(kernel)


def host_info():
    """CPU model, the cores this process may run on and the BLAS thread pools."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()
                if d.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_baseline(scene, nrhs, budget_s=15.0, max_rows=512):
    """FP64 oracle: dense rows of eq. (4) assembled for a random row sample (as many as
    the budget allows, at least 4), then the dense product of that row block with all
    right-hand sides timed and scaled to a full N-row product."""
    import numpy as np

    import oracle
    from oracle import dense
    p = oracle.panelize(scene["cond_id"], scene["eps_r"], scene["eps_b"])
    N = len(p["axis"])
    rng = np.random.default_rng(0)
    order = rng.permutation(N)[:min(N, max_rows)]
    blocks = []
    t0 = time.perf_counter()
    done = 0
    while done < len(order):
        step = min(8, len(order) - done)
        rows = np.sort(order[done:done + step])
        blocks.append((rows, dense.assemble_rows(p, rows)))
        done += step
        if time.perf_counter() - t0 > budget_s and done >= 4:
            break
    t_asm = time.perf_counter() - t0
    A = np.concatenate([b for _, b in blocks], axis=0)
    nrow = A.shape[0]
    X = rng.standard_normal((N, nrhs))
    reps = 0
    t0 = time.perf_counter()
    while True:
        A @ X
        reps += 1
        el = time.perf_counter() - t0
        if el > 5.0 or reps >= 2000:
            break
    t_block = el / reps
    t_full = t_block * N / nrow
    h = host_info()
    return {"value": nrhs / t_full, "unit": "RHS-MVPs/s", "cores": h["cores"], "kind": "oracle",
            "sample": (f"{nrow} random rows of the dense eq.(4) matrix (N={N}) assembled by the oracle in "
                       f"{t_asm:.1f}s ({t_asm / nrow * N:.0f}s extrapolated to all rows, not counted), "
                       f"row-block product with {nrhs} RHS timed over {reps} reps and scaled by N/rows"),
            "assembly_s_per_row": t_asm / nrow, "cpu_model": h["cpu_model"], "blas": h["blas"]}


# scenes of the oracle timing table: the two dense-solvable workloads at full size and
# the three larger ones scaled down by the same seeded generators
ORACLE_TABLE = [
    ("cube16", lambda sc: sc.cube(16, 1.0)),
    ("plates", lambda sc: sc.parallel_plates()),
    ("random128/4 (32^3, 8 conductors, 6 dielectric boxes)",
     lambda sc: sc.random_boxes(n=32, edge=(2, 6))),
    ("meander/8 (64x64x16, 4 lanes, 2 runs)",
     lambda sc: sc.meander(nx=64, ny=64, runs=2, run_pitch=24, x0=8, x1=48)),
    ("grad256/5 (48x48x16, 6 conductors, 16 blocks)",
     lambda sc: sc.gradient_scene(nx=48, ny=48, nz=16, sub=(2, 14))),
]


def oracle_table():
    """The FP64 oracle's dense route on this host: assembly of eq. (4), LU factorisation
    and one dense product with all right-hand sides, per scene (no GPU)."""
    import numpy as np

    import oracle
    import scenes
    from oracle import dense
    out = {"host": host_info(), "rows": []}
    for name, make in ORACLE_TABLE:
        s = make(scenes)
        p = oracle.panelize(s["cond_id"], s["eps_r"], s["eps_b"])
        N = len(p["axis"])
        t0 = time.perf_counter()
        A = dense.assemble(p)
        t_asm = time.perf_counter() - t0
        B = dense.rhs(p)
        t0 = time.perf_counter()
        rho, lu = dense.solve(A, B)
        t_lu = time.perf_counter() - t0
        reps, t0 = 0, time.perf_counter()
        while True:
            A @ B
            reps += 1
            if time.perf_counter() - t0 > 2.0:
                break
        t_mvp = (time.perf_counter() - t0) / reps
        row = {"scene": name, "grid": list(s["cond_id"].shape), "N": N, "m": int(p["m"]),
               "assembly_s": t_asm, "lu_solve_s": t_lu, "dense_mvp_s": t_mvp,
               "rhs_mvps_per_s": p["m"] / t_mvp, "dense_gflops": 2.0 * N * N * p["m"] / t_mvp / 1e9}
        out["rows"].append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del A, lu
    print(json.dumps(out), flush=True)


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
    # the y pass runs on one of three kernels (the autotuner's choice; the register-edge
    # kernel with one or two columns per thread): the timed steps' y launches are the
    # last 2 x steps of them, alternating forward / inverse
    kern = {"zfwd_scatter": ("k_zfwd<" + tname,),
            "y": ("k_strided<" + tname, "k_ypass<" + tname, "k_ypass_n<" + tname),
            "x_sandwich_multiply": ("k_xsandwich<" + tname, "k_xsandwich_tk<" + tname),
            "zinv_gather": ("k_zinv<" + tname,)}

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
    tk = "" if args.tucker_tol is None else f" --tucker-tol {args.tucker_tol:g}"
    cmd = (f"python bench.py --config {args.config} --prec {args.prec} --steps {args.steps} --warmup {args.warmup} "
           f"--no-cpu --no-solve --no-other{tk} --toeplitz-tol 0 --batch 0 --calib-copy-mib {args.calib_copy_mib}")
    res = {"source_hash": kernel_source_hash(), "config": args.config, "prec": args.prec,
           "tucker_tol": WORKLOAD_TUCKER.get(args.config, 0.0) if args.tucker_tol is None else args.tucker_tol,
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


def tucker_summary(P, prec, ms_step, ms_step_plain, rb_ms, x_ms, nrhs):
    """Tucker form of the step's spectra (eq. 13), never stored whole: ranks, compression
    ratio, the bytes resident, the strips' rebuild (T1 = S x3 U3, T2 = T1 x2 U2, two
    batched MFMA GEMMs) with its MFMA rate, the x-mode product X = U1 T2 that the x pass
    forms per tile on the matrix cores (its flops and their rate over the x pass), and
    the paper's computational overhead CO, here the Tucker step's extra time over the
    uncompressed product divided by that product."""
    info = P.tucker_info()
    Mx, My, Mz = P.fft_size()
    D = (Mx // 2 + 1, My // 2 + 1, Mz // 2 + 1)
    flops = 0.0
    out_bytes = 0.0
    xmode = 0.0
    elem = 4 if prec == "fp32" else 8
    for r1, r2, r3 in info["ranks"]:
        r1p = (r1 + 3) // 4 * 4
        flops += 2.0 * (r1 * r2 * r3 * D[2] + r1 * r2 * D[1] * D[2])
        out_bytes += elem * (r1 * r2 * D[2] + r1p * D[1] * D[2])        # T1 and T2 written
        # per (ky, kz) column of the x pass (all My * H of them, once per tile)
        xmode += 2.0 * D[0] * r1 * My * D[2]
    tf = flops / (rb_ms / 1e3) / 1e12 if rb_ms > 0 else None
    xtf = xmode / (x_ms / 1e3) / 1e12 if x_ms > 0 else None
    return {"ranks": info["ranks"], "compression_ratio": info["compression_ratio"],
            "spectra_bytes_resident": P.spectra_bytes(),
            "step_ms": ms_step, "uncompressed_step_ms": ms_step_plain,
            "computational_overhead": (ms_step - ms_step_plain) / ms_step_plain if ms_step_plain else None,
            "strip_rebuild": {"ms": rb_ms, "flops": flops, "achieved_tflops": tf,
                              "mfma_frac": tf / MFMA_PEAK_TFLOPS[prec] if tf else None,
                              "bytes_written": out_bytes,
                              "achieved_gbs": out_bytes / (rb_ms / 1e3) / 1e9 if rb_ms > 0 else None},
            "xmode_in_x_pass": {"flops_per_launch": xmode, "x_pass_ms": x_ms,
                                "tflops_over_x_pass": xtf,
                                "mfma_frac_over_x_pass": xtf / MFMA_PEAK_TFLOPS[prec] if xtf else None}}


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


# Tucker tolerance of each workload's step (the meander lines are specified compressed)
WORKLOAD_TUCKER = {"meander": 1e-8}


def timed_products(P, x, y, prec, stream, steps, warm, level, every=1):
    """Warm-up, then `steps` products bracketed by two events (level 2: HIP events around
    the x pass on every `every`-th step; level 1: around every pass)."""
    import torch
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
    return e0.elapsed_time(e1), P.pass_times()


def solve_times(Pm, P64, log):
    """C-matrix solve times: mixed precision on the step's problem (Pm) and FP64 plain on
    the uncompressed one (P64), both at the loosest GMRES tolerance at which every gated
    entry of C is within 1e-6 of the FP64 solve at rtol 1e-12, and at rtol 1e-9."""
    import numpy as np
    import torch
    Cref, _ = P64.capacitance(prec="fp64", rtol=1e-12)
    gate = np.abs(Cref) >= 1e-3 * np.abs(np.diag(Cref)).max()

    def cerr(Cm):
        return float((np.abs(Cm - Cref)[gate] / np.abs(Cref)[gate]).max())

    def timed(P, mode, rtol, form="auto"):
        """Median of three warm solves (the restart-cycle graphs are captured by a first,
        untimed solve), with the entrywise error of the last against FP64 at 1e-12."""
        kw = {"mixed_form": form} if mode == "mixed" else {}
        P.capacitance(prec=mode, rtol=rtol, **kw)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Cm, st = P.capacitance(prec=mode, rtol=rtol, **kw)
            ts.append(time.perf_counter() - t0)
        r = {"time_s": float(np.median(ts)), "times_s": ts, "iters": st["iters"], "ir_steps": st["ir_steps"],
             "max_rel_err_vs_fp64_1e-12": cerr(Cm), "products": st["mvp_count"], "rtol": rtol,
             "spectra_bytes": st["spectra_bytes"]}
        if mode == "mixed":
            r["mixed_form"] = st["mixed_form"]
            r["steps_fp32"] = st["steps_fp32"]
        return r

    runs = (("fp64", P64), ("mixed", Pm))
    cal = 1e-10
    for rt in (1e-5, 1e-6, 1e-7, 1e-8, 1e-9):
        if all(cerr(P.capacitance(prec=mode, rtol=rt)[0]) <= 1e-6 for mode, P in runs):
            cal = rt
            break
    out = {"rtol_for_1e-6": cal, "mixed_spectra": "tucker" if Pm is not P64 else "uncompressed"}
    for mode, P in runs:
        out[mode] = timed(P, mode, cal)
        log(f"# solve {mode} at rtol {cal:g}: {out[mode]['time_s'] * 1e3:.1f} ms, "
            f"err {out[mode]['max_rel_err_vs_fp64_1e-12']:.1e}")
    out["speedup_mixed_vs_fp64"] = out["fp64"]["time_s"] / out["mixed"]["time_s"]
    out["at_rtol_1e-9"] = {mode: timed(P, mode, 1e-9) for mode, P in runs}
    out["at_rtol_1e-9"]["speedup_mixed_vs_fp64"] = (out["at_rtol_1e-9"]["fp64"]["time_s"] /
                                                    out["at_rtol_1e-9"]["mixed"]["time_s"])
    # both mixed forms explicitly ("mixed" above is the automatic choice)
    out["mixed_forms"] = {}
    for form in ("refinement", "relaxed"):
        for rt in (cal, 1e-9):
            r = timed(Pm, "mixed", rt, form)
            out["mixed_forms"][f"{form}_rtol_{rt:g}"] = {k: r[k] for k in (
                "time_s", "iters", "ir_steps", "steps_fp32", "max_rel_err_vs_fp64_1e-12")}
            log(f"# solve mixed/{form} at rtol {rt:g}: {r['time_s'] * 1e3:.2f} ms, iters {r['iters']}, "
                f"fp32 steps {r['steps_fp32']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P64.capacitance(prec="fp64", rtol=cal, graph=False)
    out["fp64_no_graph_time_s"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="meander", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="heuristic x-pass configuration instead of the autotuner")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the uncompressed and other-precision product rates")
    ap.add_argument("--batch", type=int, default=32,
                    help="also solve this many uneven random scenes (edges 16-64) as one packed set and one by one "
                         "(0: skip)")
    ap.add_argument("--tucker-tol", type=float, default=None,
                    help="Tucker tolerance of the step's spectra (default: the workload's, 1e-8 for meander, "
                         "else uncompressed; 0: uncompressed)")
    ap.add_argument("--toeplitz-tol", type=float, default=1e-8,
                    help="also build a Toeplitz cache over a larger grid at this tolerance and set the workload up "
                         "from it (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (HBM-counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="(no GPU) turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this command with "
                         "--calib-copy-mib into profiles/traffic_<config>_<prec>.json, then exit")
    ap.add_argument("--oracle-table", action="store_true",
                    help="(no GPU) time the FP64 oracle's assembly, LU and dense product on this host, then exit")
    ap.add_argument("--solve-once", choices=["mixed", "fp64"],
                    help="set the workload up, run one untimed and one timed capacitance solve in this precision "
                         "(rtol --solve-rtol), print its time and iterations as one JSON line, then exit (the last "
                         "solve of the run is the timed one, e.g. for a kernel trace)")
    ap.add_argument("--solve-rtol", type=float, default=1e-7)
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args)
        return
    if args.oracle_table:
        oracle_table()
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is design-only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2004_02609_amd import voxcap

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tucker_tol = WORKLOAD_TUCKER.get(args.config, 0.0) if args.tucker_tol is None else args.tucker_tol
    scene = scenes.by_name(args.config)
    t0 = time.perf_counter()
    P = voxcap.Problem.from_scene(scene).setup(autotune=not args.no_tune, tucker_tol=tucker_tol)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    B, N = P.m, P.N
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev).manual_seed(0)
    x = torch.randn(B, N, dtype=torch.float64, device=dev, generator=g)
    y = torch.empty_like(x)
    log(f"# {args.config}: N={N} m={B} fft={P.fft_size()} tucker_tol={tucker_tol:g} setup {t_setup:.2f}s")
    if args.solve_once:
        P.capacitance(prec=args.solve_once, rtol=args.solve_rtol)   # captures the cycle graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = P.capacitance(prec=args.solve_once, rtol=args.solve_rtol)
        torch.cuda.synchronize()
        print(json.dumps({"config": args.config, "prec": args.solve_once, "rtol": args.solve_rtol,
                          "time_s": time.perf_counter() - t0, "iters": st["iters"], "ir_steps": st["ir_steps"],
                          "mixed_form": st["mixed_form"], "steps_fp32": st["steps_fp32"]}), flush=True)
        return

    # the step: timed with events around the x pass on every `every`-th step
    every = max(1, min(10, args.steps // 10))
    ms, (pms, pcnt, pbytes) = timed_products(P, x, y, args.prec, stream, args.steps, args.warmup, 2, every)
    value = args.steps * B / (ms / 1e3)
    log(f"# step ({args.prec}{', Tucker rebuild' if tucker_tol > 0 else ''}): {ms / args.steps * 1e3:.1f} us")
    # per-pass breakdown (and the Tucker rebuild's time): a separate, shorter run with
    # events around every pass
    nb = max(10, min(args.steps, 50))
    tk0 = P.tucker_info() if tucker_tol > 0 else None
    _, (bms, bcnt, bbytes) = timed_products(P, x, y, args.prec, stream, nb, 2, 1)
    passes = {voxcap.PASS_NAMES[i]: {"avg_us": bms[i] / max(1, bcnt[i]) * 1e3, "launches": bcnt[i],
                                     "alg_bytes": bbytes[i],
                                     "alg_GBs": bbytes[i] / (bms[i] / max(1, bcnt[i]) / 1e3) / 1e9
                                     if bms[i] > 0 else None}
              for i in range(5)}
    tucker = None
    if tucker_tol > 0:
        tk1 = P.tucker_info()
        n_rb = tk1["rebuilds"] - tk0["rebuilds"]
        tucker = {"tol": tucker_tol, "strip_rebuild_ms": (tk1["rebuild_ms"] - tk0["rebuild_ms"]) / max(1, n_rb),
                  "rebuilds_timed": n_rb}

    # the uncompressed problem: FP32 rate without the rebuild, the FP64-plain rate and
    # the FP64-plain solves
    P64 = P
    rates = {}
    if tucker_tol > 0 and not (args.no_other and args.no_solve):
        P64 = voxcap.Problem.from_scene(scene).setup(autotune=not args.no_tune)
    if not args.no_other:
        for prec in ("fp32", "fp64"):
            if P64 is P and prec == args.prec:
                rates[prec] = value
                continue
            n2 = max(10, args.steps // 2)
            ms2, _ = timed_products(P64, x, y, prec, stream, n2, 3, 0)
            rates[prec] = n2 * B / (ms2 / 1e3)
            log(f"# uncompressed {prec} product: {ms2 / n2 * 1e3:.1f} us/step")

    xi = voxcap.PASS_NAMES.index("x_sandwich_multiply")
    # the x pass does ~30 flops per algorithmic byte (nine transforms per column) and is
    # bound by vector-instruction issue, not HBM: report it against the vector peak
    nout = 6 if P.n_diel > 0 else 3
    x_ms = pms[xi] / max(1, pcnt[xi])
    x_flops = xpass_flops(P.fft_size(), B, nout)
    x_tflops = x_flops / (x_ms / 1e3) / 1e12
    x_traffic = load_traffic(args.config, "x_sandwich_multiply", args.prec, tucker_tol)
    roofline = {"bound": "alu", "kernel": "x_sandwich_multiply", "achieved": x_tflops,
                "peak": VEC_PEAK_TFLOPS[args.prec], "unit": "TFLOP/s", "frac": x_tflops / VEC_PEAK_TFLOPS[args.prec],
                "traffic": x_traffic, "alg_flops": x_flops, "alg_bytes": pbytes[xi], "avg_us": x_ms * 1e3,
                "hbm_achieved_GBs": pbytes[xi] / (x_ms / 1e3) / 1e9,
                "hbm_frac": pbytes[xi] / (x_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                "timed_launches": pcnt[xi], "event_sampling": f"every {every}th of the {args.steps} timed steps"}
    dom = int(np.argmax(bms))
    avg_ms = bms[dom] / max(1, bcnt[dom])
    achieved = bbytes[dom] / (avg_ms / 1e3) / 1e9
    kname = voxcap.PASS_NAMES[dom]

    if tucker is not None:
        ms_plain = B / rates[args.prec] * 1e3 if args.prec in rates else None
        tucker.update(tucker_summary(P, args.prec, ms / args.steps, ms_plain, tucker["strip_rebuild_ms"], x_ms, B))

    solve = None
    if not args.no_solve:
        solve = solve_times(P, P64, log)

    toeplitz = None
    if args.toeplitz_tol > 0:
        toeplitz = toeplitz_run(args, scene, x)

    batch = None
    if args.batch > 0:
        batch = batch_run(args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(scene, B)

    form = f"FP32 FFT product{' with Tucker-%g spectra rebuilt each step' % tucker_tol if tucker_tol > 0 else ''}"
    line = {
        "metric": "FFT-MVPs/s + C-matrix solve time @1e-6 rel err, mixed/batched vs FP64 plain",
        "value": value, "unit": "RHS-MVPs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "panels": N, "rhs": B,
                   "fft_size": list(P.fft_size()), "product_precision": args.prec, "tucker_tol": tucker_tol,
                   "step": form if args.prec == "fp32" else form.replace("FP32", "FP64")},
        "roofline": roofline,
        "product_hbm": {"dominant_pass": kname, "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS,
                        "traffic": load_traffic(args.config, kname, args.prec, tucker_tol),
                        "all_passes_alg_bytes": float(sum(bbytes)),
                        "all_passes_GBs": float(sum(bbytes)) / (ms / args.steps / 1e3) / 1e9},
        "cpu_baseline": cpu,
        "uncompressed_rates": {p: {"value": v, "unit": "RHS-MVPs/s"} for p, v in rates.items()},
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
