#!/usr/bin/env python3
"""Benchmark of the Dirac matrix times a block of N_v vectors on one MI355X.

Headline (one JSON line on stdout): Wilson D_W at c_SW = 0 on a 16^3 x 32
lattice, N_v = 12 right-hand sides, m0 = 0.1, FP32, exp(0.3 i H) links --
Gflop/s at the standard 1320 flops per site and right-hand side, and the
kernel's share of the HBM bandwidth roofline.  A step is one application of
D_W to the 12-vector block (site indexing, 8 hops with spin projection,
single write of every output).  Inputs are resident in HBM before timing;
R rotating (U, in, out) sets (default 4, about 1.4 GB) keep the working set
well above the 256 MB Infinity Cache.  Each operator row is launched through
the C ABI with its arguments marshalled once, and runs untimed for 0.1 s
before its W warmup and K timed launches (the first tens of milliseconds of
back-to-back launches are slower while the clocks settle).  ``us`` is the mean
over the K launches between two events; ``us_median_single`` the median of 50
further launches, each between its own pair of events.

Further rows (``rows`` in the JSON line), each timed the same way:
D_S 32^4 and 8^4, D_B 32^4 (FP32, FP64) with its W construction, D_W in
BF16 storage, D_W and D_B with the clover term (c_SW = 1), D_W and D_S with
compressed links (two stored rows per link) against full links, D_B with W
built on the fly from V inside the kernel, link gradients at 24^3 x 48 (D_S,
D_W, and D_B with respect to W and through W to V), and the mixed-precision
solve at 32^3 x 64 (time to
||b - D x|| / ||b|| <= 1e-10 with FP32, BF16 and FP16 inner storage, on the
full lattice and on the even-odd Schur complement).

cpu_baseline: the FP64 numpy oracle applying the same operator on the host
cores (BLAS pinned to one thread), on the full headline workload, with the
host's CPU model and thread environment variables.  With the rows, the
oracle's CGNR on an 8^4 lattice (two right-hand sides) is timed beside the GPU
solve of the same system.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import statistics
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK = 157.3e12      # MI355X FP32 vector (plain FMA, no packed instructions, measured at 115-125)
FP64_VALU_PEAK = 78.6e12       # MI355X FP64 vector
FLOPS = {"staggered": 570, "wilson": 1320, "brillouin": 28224}   # per site and right-hand side
CLOVER_FLOPS = 576             # two 6x6 complex matrix-vector products and their addition, per site and rhs

# The mixed-precision solve of D_W x = b on 32^3 x 64, N_v = 12, m0 = 0.05 to
# ||b - D x|| / ||b|| <= 1e-10: inner storage and inner tolerance of each timed
# solve, full lattice and even-odd (the fastest setting of a sweep over the
# inner tolerance on this system for each storage).
SOLVE_DIMS, SOLVE_NV, SOLVE_M0, SOLVE_TOL = (32, 32, 32, 64), 12, 0.05, 1e-10
SOLVE_SETTINGS = {
    "full": (("c64", 3e-4), ("bf16", 0.02), ("f16", 2e-3)),
    "eo": (("c64", 3e-4), ("bf16", 5e-3), ("f16", 5e-3)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def site_bytes(op: str, nv: int, eb: int, compressed: bool = False) -> int:
    """Compulsory bytes per site: links read once, input read once, output written once
    (compressed links: two of the three rows of each)."""
    links = {"staggered": 36, "wilson": 36, "brillouin": 360}[op] * (2 if compressed else 3) // 3
    comps = 3 if op == "staggered" else 12
    return eb * (links + 2 * comps * nv)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dslash_common.hpp", "stencils.hpp", "rows.hpp", "tiles.hpp", "apply.hip", "apply_rows.hip"):
        with open(os.path.join(ROOT, "paper_1808_05506_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(name)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


SETTLE_SECONDS = 0.1


def settle(torch, launch, seconds: float = SETTLE_SECONDS) -> int:
    """Untimed launches for ``seconds`` of wall time before the warmup steps: the
    first tens of milliseconds of back-to-back launches run measurably slower
    (clock and power ramp), which a short warmup does not cover.  Returns the
    number of launches."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            launch(n)
            n += 1
        torch.cuda.synchronize()
    return n


def timed(torch, launch, steps: int, warmup: int) -> float:
    """Mean seconds per launch over ``steps`` launches on the current stream."""
    for i in range(warmup):
        launch(i)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(steps):
        launch(i)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def median_single(torch, launch, count: int = 50) -> float:
    """Median seconds of ``count`` launches, each between its own pair of events
    on the current stream (enqueued back to back, so the GPU does not idle)."""
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    for i, (a, b) in enumerate(ev):
        a.record(st)
        launch(i)
        b.record(st)
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev) / 1e3


def rotated_sets(torch, U, P, count: int, C=None):
    """``count`` distinct input sets: lattice translations of (U, P[, C]) along t."""
    roll = lambda x, k: None if x is None else torch.roll(x, shifts=k, dims=0).contiguous()  # noqa: E731
    sets = [(U, P, C)]
    for k in range(1, count):
        sets.append((roll(U, k), roll(P, k), roll(C, k)))
    return sets


def abi_launcher(torch, D, op, U, P, out, mass, clover=None, compressed=False):
    """A closure that enqueues one application through the C ABI with its
    arguments marshalled once (the Python binding's per-call checks cost about
    as much host time as the kernel takes on the GPU, which would leave the
    GPU idle between back-to-back launches)."""
    import ctypes
    D.apply(op, U, P, mass, out=out, clover=clover) if not compressed else D.apply_compressed(op, U, P, mass, out=out)
    lib = D._lib
    code = D.op_code(op)
    nt, nz, ny, nx = P.shape[:4]
    dims = (ctypes.c_int * 4)(nx, ny, nz, nt)
    nv = P.shape[-1] if P.dtype in (torch.complex64, torch.complex128) else P.shape[-2]
    dt = D._dtype_code(P)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vu, vp, vo = ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(out.data_ptr())
    m = ctypes.c_double(mass)
    if compressed:
        fn, args = lib.dslash_apply_compressed, (code, vu, vp, vo, dims, 3, nv, m, 0, dt, stream)
    elif clover is not None:
        fn, args = lib.dslash_apply_clover, (code, vu, ctypes.c_void_p(clover.data_ptr()), vp, vo, dims, 3, nv, m, 0,
                                             dt, stream)
    else:
        fn, args = lib.dslash_apply, (code, vu, vp, vo, dims, 3, nv, m, dt, stream)

    def launch():
        rc = fn(*args)
        if rc:
            raise RuntimeError(f"{fn.__name__} failed: {rc}")
    return launch


def bench_apply(torch, D, op, U, P, mass, steps, warmup, rotate, dtype_bytes, label, clover=None, compressed=False):
    sets = rotated_sets(torch, U, P, rotate, clover)
    outs = [torch.empty_like(P) for _ in sets]
    launchers = [abi_launcher(torch, D, op, u, p, o, mass, c, compressed) for (u, p, c), o in zip(sets, outs)]
    launch = lambda i: launchers[i % len(launchers)]()  # noqa: E731
    settle(torch, launch)
    t = timed(torch, launch, steps, warmup)
    t_med = median_single(torch, launch)
    nt, nz, ny, nx = P.shape[:4]
    vol = nt * nz * ny * nx
    nv = P.shape[-1] if P.dtype in (torch.complex64, torch.complex128) else P.shape[-2]
    flops = (FLOPS[op] + (CLOVER_FLOPS if clover is not None else 0)) * vol * nv
    nbytes = (site_bytes(op, nv, dtype_bytes, compressed) + (36 * dtype_bytes if clover is not None else 0)) * vol
    row = {"us": t * 1e6, "us_median_single": t_med * 1e6, "gflops": flops / t / 1e9, "gbs": nbytes / t / 1e9,
           "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": nbytes, "flops_per_launch": flops,
           "dims": [nx, ny, nz, nt], "nv": nv, "rotate": rotate}
    log(f"{label}: {t * 1e6:.1f} us  {row['gflops']:.0f} Gflop/s  {row['gbs']:.0f} GB/s")
    return row, t


def launch_row(torch, launch, steps, warmup, nbytes, rotate, label, single=50):
    """Time ``launch`` as the operator rows are timed: settle, warmup, mean over
    ``steps`` launches, median of ``single`` single launches."""
    settle(torch, launch)
    t = timed(torch, launch, steps, warmup)
    t_med = median_single(torch, launch, single)
    log(f"{label}: {t * 1e6:.1f} us (median single {t_med * 1e6:.1f} us), {nbytes / t / 1e9:.0f} GB/s")
    return {"us": t * 1e6, "us_median_single": t_med * 1e6, "gbs": nbytes / t / 1e9,
            "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": nbytes, "rotate": rotate}


def solve_oracle_baseline(torch, D, np, synthetic, nv: int = 2):
    """The oracle's FP64 CGNR for D_W x = b on 8^4, m0 = 0.05, smooth links
    (seed 3), b the first nv of the 12 right-hand sides of seed 103 (a bounded
    sample: all 12 take over a minute on one core), to a normal-equation
    residual of 1e-10 with BLAS on one thread, beside the GPU solve of the same
    system (FP32 inner CG, FP64 defect correction to ||b - D x|| / ||b|| <= 1e-10)."""
    from threadpoolctl import threadpool_limits

    from oracle import solver, wilson
    dims, m0 = (8, 8, 8, 8), 0.05
    u = synthetic.gauge_links(dims, "smooth", 3)
    b = np.ascontiguousarray(synthetic.wilson_spinor(dims, 12, 103)[..., :nv])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        x, iters, _ = solver.cgnr(lambda v: wilson.apply(u, v, m0), lambda v: wilson.apply(u, v, m0, True), b,
                                  tol=1e-10)
        t_oracle = time.perf_counter() - t0
    true_res = float(np.max(solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, x)))
    U = torch.from_numpy(u).cuda()
    B = torch.from_numpy(b).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xg, info = D.solve("wilson", U, B, m0, inner="c64", tol=1e-10, inner_tol=1e-5)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    log(f"solve 8^4 N_v={nv}: oracle CGNR {t_oracle:.1f} s ({int(np.max(iters))} iterations, relres {true_res:.1e}), "
        f"GPU {t_gpu:.3f} s")
    return {"oracle_seconds": t_oracle, "oracle_iters": int(np.max(iters)), "oracle_relres": true_res,
            "oracle_cores": 1, "gpu_seconds": t_gpu, "gpu_inner_iters": info["inner_iters"],
            "gpu_max_relres": max(info["relres"]), "dims": list(dims), "nv": nv, "m0": m0,
            "sample": f"the first {nv} of the 12 right-hand sides"}


def cpu_baseline(dims, nv, m0, min_seconds: float = 10.0):
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synthetic
    from oracle import wilson
    u = synthetic.round_to(synthetic.gauge_links(dims, "smooth", 1), "c64")
    p = synthetic.round_to(synthetic.wilson_spinor(dims, nv, 101), "c64")
    vol = int(np.prod(dims))
    reps, t_total = 0, 0.0
    with threadpool_limits(limits=1):
        while t_total < min_seconds and reps < 5:
            t0 = time.perf_counter()
            wilson.apply(u, p, m0)
            t_total += time.perf_counter() - t0
            reps += 1
    gflops = FLOPS["wilson"] * vol * nv * reps / t_total / 1e9
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads_env = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
                   if k in os.environ}
    return {"value": gflops, "unit": "Gflop/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model,
            "threads_env": threads_env,
            "sample": f"{reps} full FP64 numpy applications of D_W (eq. def_wils, literal form) to the same "
                      f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} N_v={nv} workload, {t_total:.1f} s, BLAS pinned to 1 thread",
            "host_cpus": len(os.sched_getaffinity(0))}


def staggered_rows_bench(torch, D, np, synthetic, steps, warmup):
    """The D_S rows: 8^4, N_v = 4 (cache-resident, launch-bound) and 32^4, N_v = 12."""
    rows = {}
    dev = torch.device("cuda:0")

    def up(a, dt):
        return torch.from_numpy(a.astype(dt)).to(dev)

    u = synthetic.gauge_links((8, 8, 8, 8), "haar", 0)
    p = synthetic.staggered_spinor((8, 8, 8, 8), 4, 100)
    rows["staggered_8^4_nv4_fp32"], _ = bench_apply(torch, D, "staggered", up(u, np.complex64), up(p, np.complex64),
                                                    0.0, steps, warmup, 1, 8, "D_S 8^4 nv4")
    dims = (32, 32, 32, 32)
    U = up(synthetic.gauge_links(dims, "haar", 0), np.complex64)
    P = up(synthetic.staggered_spinor(dims, 12, 100), np.complex64)
    rows["staggered_32^4_nv12_fp32"], _ = bench_apply(torch, D, "staggered", U, P, 0.0, steps, warmup, 1, 8,
                                                      "D_S 32^4 nv12")
    del U, P
    torch.cuda.empty_cache()
    return rows


def block_size_rows_bench(torch, D, np, synthetic, steps, warmup):
    """D_W on the headline lattice (16^3 x 32, FP32, smooth links seed 1, rhs
    seed 101) at other block sizes N_v: 4, 8, 16 and 24 take the row-staged
    t-marching kernel, N_v = 1 the direct one; D_S and D_B on 32^4 (FP32) at
    N_v = 4 and 24."""
    rows = {}
    dev = torch.device("cuda:0")
    dims = (16, 16, 16, 32)
    U = torch.from_numpy(synthetic.gauge_links(dims, "smooth", 1).astype(np.complex64)).to(dev)
    for nv in (1, 4, 8, 16, 24):
        P = torch.from_numpy(synthetic.wilson_spinor(dims, nv, 101).astype(np.complex64)).to(dev)
        rows[f"wilson_16^3x32_nv{nv}_fp32"], _ = bench_apply(torch, D, "wilson", U, P, 0.1, steps, warmup, 4, 8,
                                                             f"D_W 16^3x32 nv{nv} fp32")
        del P
    del U
    dims = (32, 32, 32, 32)
    U = torch.from_numpy(synthetic.gauge_links(dims, "haar", 0).astype(np.complex64)).to(dev)
    for nv in (4, 24):
        P = torch.from_numpy(synthetic.staggered_spinor(dims, nv, 100).astype(np.complex64)).to(dev)
        rows[f"staggered_32^4_nv{nv}_fp32"], _ = bench_apply(torch, D, "staggered", U, P, 0.0, steps, warmup, 1, 8,
                                                             f"D_S 32^4 nv{nv} fp32")
        del P
    del U
    # D_B on 32^4 (FP32, Haar links seed 2, W built on the GPU untimed, rhs seed 102)
    W = D.brillouin_links(torch.from_numpy(synthetic.gauge_links(dims, "haar", 2).astype(np.complex64)).to(dev))
    for nv in (4, 24):
        P = torch.from_numpy(synthetic.wilson_spinor(dims, nv, 102).astype(np.complex64)).to(dev)
        row, t = bench_apply(torch, D, "brillouin", W, P, 0.1, max(3, steps // 10), 2, 1, 8, f"D_B 32^4 nv{nv} fp32")
        row["valu_frac"] = row["flops_per_launch"] / t / FP32_VALU_PEAK
        rows[f"brillouin_32^4_nv{nv}_fp32"] = row
        del P
    del W
    torch.cuda.empty_cache()
    return rows


def brillouin_rows_bench(torch, D, np, synthetic, steps, fly=False):
    """The D_B rows on 32^4, N_v = 12: FP32 and FP64 with the W construction
    time, and (fly) the clover term and W built on the fly in FP32."""
    rows = {}
    dev = torch.device("cuda:0")

    def up(a, dt):
        return torch.from_numpy(a.astype(dt)).to(dev)

    dims = (32, 32, 32, 32)
    # D_B 32^4, N_v = 12, FP32 and FP64 (W built on the GPU, untimed setup)
    v = synthetic.gauge_links(dims, "haar", 2)
    p = synthetic.wilson_spinor(dims, 12, 102)
    for name, cdt, eb, peak in (("fp32", np.complex64, 8, FP32_VALU_PEAK), ("fp64", np.complex128, 16, FP64_VALU_PEAK)):
        V = up(v, cdt)
        t0 = time.perf_counter()
        W = D.brillouin_links(V)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        del V
        P = up(p, cdt)
        row, t = bench_apply(torch, D, "brillouin", W, P, 0.1, max(3, steps // 10), 2, 1, eb, f"D_B 32^4 {name}")
        row["valu_frac"] = row["flops_per_launch"] / t / peak
        row["valu_peak_tflops"] = peak / 1e12
        row["w_build_ms"] = tw * 1e3
        rows[f"brillouin_32^4_nv12_{name}"] = row
        if name == "fp32" and fly:
            # with the clover term (c_SW = 1), built from V on the GPU (untimed setup)
            V = up(v, cdt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C = D.clover_field(V, 1.0)
            torch.cuda.synchronize()
            tc = time.perf_counter() - t0
            del V
            row, t = bench_apply(torch, D, "brillouin", W, P, 0.1, max(3, steps // 10), 2, 1, eb,
                                 "D_B + clover 32^4 fp32", clover=C)
            row["valu_frac"] = row["flops_per_launch"] / t / peak
            row["clover_build_ms"] = tc * 1e3
            row["c_sw"] = 1.0
            rows["brillouin_clover_32^4_nv12_fp32"] = row
            del C
            # the same operator with W built on the fly from V inside the kernel (no W array)
            V = up(v, cdt)
            sets_v = [V]

            def fly(i):
                D.apply_brillouin_fly(sets_v[0], P, 0.1, out=out_fly)
            out_fly = torch.empty_like(P)
            nfly = max(3, steps // 10)
            tf = timed(torch, fly, nfly, 2)
            vol = int(np.prod(dims))
            fbytes = (36 + 2 * 12 * 12) * eb * vol
            rows["brillouin_fly_32^4_nv12_fp32"] = {
                "us": tf * 1e6, "gflops": FLOPS["brillouin"] * vol * 12 / tf / 1e9,
                "valu_frac": FLOPS["brillouin"] * vol * 12 / tf / peak, "gbs": fbytes / tf / 1e9,
                "bytes_per_launch": fbytes, "vs_stored_w": rows["brillouin_32^4_nv12_fp32"]["us"] / (tf * 1e6),
                "note": "apply flops only (the W construction inside the kernel is not counted)"}
            log(f"D_B fly 32^4 fp32: {tf * 1e6:.1f} us")
            del V, out_fly
        del W, P
        torch.cuda.empty_cache()
    return rows


def rows_bench(torch, D, np, synthetic, steps, warmup):
    rows = {}
    dev = torch.device("cuda:0")

    def up(a, dt):
        return torch.from_numpy(a.astype(dt)).to(dev)

    rows.update(staggered_rows_bench(torch, D, np, synthetic, steps, warmup))
    rows.update(block_size_rows_bench(torch, D, np, synthetic, steps, warmup))
    rows.update(brillouin_rows_bench(torch, D, np, synthetic, steps, fly=True))
    # D_W with BF16 storage (FP32 arithmetic) on the headline workload
    dims = (16, 16, 16, 32)
    u = synthetic.gauge_links(dims, "smooth", 1)
    p = synthetic.wilson_spinor(dims, 12, 101)
    Ub = D.convert(up(u, np.complex64), "bf16")
    Pb = D.convert(up(p, np.complex64), "bf16")
    rows["wilson_16^3x32_nv12_bf16"], _ = bench_apply(torch, D, "wilson", Ub, Pb, 0.1, steps, warmup, 4, 4,
                                                      "D_W bf16")
    del Ub, Pb
    # D_W with the clover term (c_SW = 1) on the headline workload, FP32
    U, P = up(u, np.complex64), up(p, np.complex64)
    C = D.clover_field(U, 1.0)
    row, _ = bench_apply(torch, D, "wilson", U, P, 0.1, steps, warmup, 4, 8, "D_W + clover fp32", clover=C)
    row["c_sw"] = 1.0
    rows["wilson_clover_16^3x32_nv12_fp32"] = row
    # the same D_W with compressed links (two stored rows per link)
    rows["wilson_compressed_16^3x32_nv12_fp32"], _ = bench_apply(
        torch, D, "wilson", D.compress_links(U), P, 0.1, steps, warmup, 4, 8, "D_W compressed fp32", compressed=True)
    del U, P, C
    # link-dominated cases (N_v = 1) and D_S at N_v = 12, full and compressed links, 32^4
    dims = (32, 32, 32, 32)
    for op, gen, kind, seed in (("wilson", synthetic.wilson_spinor, "smooth", 1),
                                ("staggered", synthetic.staggered_spinor, "haar", 0)):
        U = up(synthetic.gauge_links(dims, kind, seed), np.complex64)
        Uc = D.compress_links(U)
        for nv in ((1, 12) if op == "staggered" else (1,)):
            P = up(gen(dims, nv, 100), np.complex64)
            mass = 0.1 if op == "wilson" else 0.0
            r_full, _ = bench_apply(torch, D, op, U, P, mass, steps, warmup, 1, 8, f"{op} 32^4 nv{nv} fp32")
            r_comp, _ = bench_apply(torch, D, op, Uc, P, mass, steps, warmup, 1, 8, f"{op} compressed 32^4 nv{nv}",
                                    compressed=True)
            r_comp["speedup_vs_full_links"] = r_full["us"] / r_comp["us"]
            rows[f"{op}_32^4_nv{nv}_fp32"] = r_full
            rows[f"{op}_compressed_32^4_nv{nv}_fp32"] = r_comp
            del P
        del U, Uc
    torch.cuda.empty_cache()
    rows.update(gradient_rows_bench(torch, D, np, synthetic, steps, warmup))
    rows.update(solve_rows_bench(torch, D, np, synthetic))
    return rows


def gradient_rows_bench(torch, D, np, synthetic, steps, warmup):
    """The link gradients at 24^3 x 48, N_v = 12, FP32, timed like the operator
    rows (settle, warmup, mean over the timed launches, median single launch);
    D_S rotates two translated (chi, psi, G) sets so the footprint exceeds 1 GB.
    Then the Brillouin ones: with respect to W, the W construction, and through
    it to V."""
    import ctypes
    rows = {}
    dev = torch.device("cuda:0")

    def up(a, dt):
        return torch.from_numpy(a.astype(dt)).to(dev)
    lib = D._lib
    dims = (24, 24, 24, 48)
    vol = int(np.prod(dims))
    dims_c = (ctypes.c_int * 4)(*dims)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    for op, kind, seed in (("staggered", "haar", 4), ("wilson", "smooth", 5)):
        gen = synthetic.staggered_spinor if op == "staggered" else synthetic.wilson_spinor
        U = up(synthetic.gauge_links(dims, kind, seed), np.complex64)
        C = up(gen(dims, 12, 104), np.complex64)
        P = up(gen(dims, 12, 105), np.complex64)
        nrot = 2 if op == "staggered" else 1
        sets = [(torch.roll(C, k, 0).contiguous(), torch.roll(P, k, 0).contiguous(), torch.empty_like(U))
                for k in range(nrot)]
        code = D.op_code(op)
        args = [(code, vp(U), vp(c), vp(p), vp(g), None, dims_c, 3, 12, 0.0, 0, stream) for c, p, g in sets]

        def launch(i, args=args):
            if lib.dslash_backward(*args[i % len(args)]):
                raise RuntimeError("dslash_backward failed")
        nbytes = site_bytes(op, 12, 8) * vol
        rows[f"link_grad_{op}_24^3x48_nv12_fp32"] = launch_row(torch, launch, steps, warmup, nbytes, nrot,
                                                               f"link grad {op}")
        del U, C, P, sets
    torch.cuda.empty_cache()
    # Brillouin link gradient at 24^3 x 48, N_v = 12, FP32: with respect to the stored W
    # (dslash_backward), then through the W construction to V: by the first-hop recursion of
    # the path averages (dslash_brillouin_links_backward_ws, the default) and by the sums over
    # the orderings through W (dslash_brillouin_links_backward)
    V = up(synthetic.gauge_links(dims, "haar", 6), np.complex64)
    W = D.brillouin_links(V)
    C = up(synthetic.wilson_spinor(dims, 12, 104), np.complex64)
    P = up(synthetic.wilson_spinor(dims, 12, 105), np.complex64)
    gW = torch.empty_like(W)
    gV = torch.empty_like(V)

    def wgrad(i):
        if lib.dslash_backward(2, vp(W), vp(C), vp(P), vp(gW), None, dims_c, 3, 12, 0.0, 0, stream):
            raise RuntimeError("dslash_backward failed")

    nws = lib.dslash_brillouin_links_backward_workspace_bytes(dims_c, 3, 0)
    ws = torch.empty(nws, dtype=torch.uint8, device=V.device)

    def vgrad(i):
        if lib.dslash_brillouin_links_backward_ws(vp(V), vp(W), vp(gW), vp(gV), vp(ws), nws, dims_c, 3, 0, stream):
            raise RuntimeError("dslash_brillouin_links_backward_ws failed")

    def vgrad_subsets(i):
        if lib.dslash_brillouin_links_backward(vp(V), vp(W), vp(gW), vp(gV), dims_c, 3, 0, stream):
            raise RuntimeError("dslash_brillouin_links_backward failed")
    nsteps = max(3, steps // 20)
    bw = (2 * 12 * 12 * 8 + 360 * 8) * vol   # chi and psi read, G_W written
    bv = (360 * 8 + 360 * 8 + 36 * 8 + 36 * 8) * vol   # W, G_W and V read, G_V written
    rows["link_grad_brillouin_W_24^3x48_nv12_fp32"] = launch_row(torch, wgrad, nsteps, 1, bw, 1,
                                                                 "Brillouin link grad (W)", single=10)
    rows["brillouin_links_backward_24^3x48_fp32"] = launch_row(torch, vgrad, nsteps, 1, bv, 1,
                                                               "Brillouin links backward (V), levels", single=10)
    Wb = torch.empty_like(W)

    def wbuild(i):
        if lib.dslash_brillouin_links(vp(V), vp(Wb), dims_c, 3, 0, stream):
            raise RuntimeError("dslash_brillouin_links failed")
    rows["brillouin_links_24^3x48_fp32"] = launch_row(torch, wbuild, nsteps, 1, (36 + 360) * 8 * vol, 1,
                                                      "Brillouin W construction", single=10)
    del Wb
    rows["brillouin_links_backward_subsets_24^3x48_fp32"] = launch_row(
        torch, vgrad_subsets, nsteps, 1, bv, 1, "Brillouin links backward (V), sums over orderings", single=5)
    del V, W, C, P, gW, gV, ws
    torch.cuda.empty_cache()
    return rows


def solve_rows_bench(torch, D, np, synthetic):
    """The mixed-precision solves of D_W x = b on 32^3 x 64, N_v = 12, m0 = 0.05,
    smooth links: wall time to ||b - D x|| / ||b|| <= 1e-10 with FP32, BF16 and
    FP16 inner storage, on the full lattice and on the even-odd Schur complement."""
    rows = {}
    dev = torch.device("cuda:0")

    def up(a, dt):
        return torch.from_numpy(a.astype(dt)).to(dev)

    dims = SOLVE_DIMS
    U = up(synthetic.gauge_links(dims, "smooth", 3), np.complex128)
    B = up(synthetic.wilson_spinor(dims, SOLVE_NV, 103), np.complex128)
    solve = {}
    for inner, itol in SOLVE_SETTINGS["full"]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = D.solve("wilson", U, B, SOLVE_M0, inner=inner, tol=SOLVE_TOL, inner_tol=itol)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        solve[inner] = {"seconds": t, "inner_iters": info["inner_iters"], "outer_iters": info["outer_iters"],
                        "max_relres": max(info["relres"]), "status": info["status"], "inner_tol": itol}
        log(f"solve inner={inner}: {t:.2f} s, {info['inner_iters']} inner / {info['outer_iters']} outer, "
            f"max relres {max(info['relres']):.2e}")
        del x
    base = solve["c64"]["seconds"]
    for k in ("bf16", "f16"):
        solve[k]["speedup_vs_fp32_inner"] = base / solve[k]["seconds"]
    rows["solve_wilson_32^3x64_nv12"] = solve
    # the same solves with the inner CG on the even-site Schur complement
    solve_eo = {}
    for inner, itol in SOLVE_SETTINGS["eo"]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = D.solve("wilson", U, B, SOLVE_M0, inner=inner, tol=SOLVE_TOL, inner_tol=itol, eo=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        solve_eo[inner] = {"seconds": t, "inner_iters": info["inner_iters"], "outer_iters": info["outer_iters"],
                           "max_relres": max(info["relres"]), "status": info["status"], "inner_tol": itol,
                           "speedup_vs_full_lattice": solve[inner]["seconds"] / t,
                           "speedup_vs_fp32_inner_full_lattice": base / t}
        log(f"solve eo inner={inner}: {t:.2f} s, {info['inner_iters']} inner / {info['outer_iters']} outer, "
            f"max relres {max(info['relres']):.2e}")
        del x
    rows["solve_wilson_eo_32^3x64_nv12"] = solve_eo
    del U, B
    torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rotate", type=int, default=4)
    ap.add_argument("--rows", choices=["all", "none", "staggered", "solve", "brillouin", "nv", "gradients"],
                    default="all",
                    help="the other rows: all, none, or only the D_S ones, the solves, the D_B ones, the D_W "
                         "ones at other block sizes N_v or the link gradients")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain FP32 complex copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic
    from paper_1808_05506_amd import dslash as D

    dims, nv, m0 = (16, 16, 16, 32), 12, 0.1
    dev = torch.device("cuda:0")
    log(f"device: {torch.cuda.get_device_name(0)}")
    copy_row = None
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.zeros(n, dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        import ctypes
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def copy(i):
            rc = D._lib.dslash_convert(ctypes.c_void_p(src.data_ptr()), 0, ctypes.c_void_p(dst.data_ptr()), 0, n, stream)
            if rc:
                raise RuntimeError(f"dslash_convert failed: {rc}")
        tc = timed(torch, copy, 10, 2)
        copy_row = {"bytes_read": n * 8, "bytes_written": n * 8, "us": tc * 1e6, "gbs": 16 * n / tc / 1e9}
        log(f"copy {args.calibrate_copy} MiB: {tc * 1e6:.1f} us, {16 * n / tc / 1e9:.0f} GB/s (read + write)")
        del src, dst
    u = synthetic.gauge_links(dims, "smooth", 1)
    p = synthetic.wilson_spinor(dims, nv, 101)
    U = torch.from_numpy(u.astype(np.complex64)).to(dev)
    P = torch.from_numpy(p.astype(np.complex64)).to(dev)
    row, t = bench_apply(torch, D, "wilson", U, P, m0, args.steps, args.warmup, args.rotate, 8, "D_W 16^3x32 nv12 fp32")
    del U, P
    torch.cuda.empty_cache()

    traffic = measured_traffic("wilson_16^3x32_nv12_fp32")
    roofline = {"bound": "hbm", "achieved": row["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": row["gbs"] / HBM_PEAK_GBS, "traffic": traffic}

    rows = {}
    if args.rows == "all":
        rows = rows_bench(torch, D, np, synthetic, args.steps, args.warmup)
    elif args.rows == "staggered":
        rows = staggered_rows_bench(torch, D, np, synthetic, args.steps, args.warmup)
    elif args.rows == "solve":
        rows = solve_rows_bench(torch, D, np, synthetic)
    elif args.rows == "brillouin":
        rows = brillouin_rows_bench(torch, D, np, synthetic, args.steps, fly=True)
    elif args.rows == "nv":
        rows = block_size_rows_bench(torch, D, np, synthetic, args.steps, args.warmup)
    elif args.rows == "gradients":
        rows = gradient_rows_bench(torch, D, np, synthetic, args.steps, args.warmup)

    cpu = None if args.no_cpu else cpu_baseline(dims, nv, m0)
    if args.rows == "all" and not args.no_cpu:
        rows["solve_wilson_8^4_oracle_vs_gpu"] = solve_oracle_baseline(torch, D, np, synthetic)

    out = {
        "metric": "Dslash Gflop/s + % HBM roofline (N_v=12, FP32); mixed-prec solve speedup",
        "value": row["gflops"],
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_seconds": SETTLE_SECONDS,
        "ms_per_step": t * 1e3,
        "ms_median_single_launch": row["us_median_single"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "wilson_dslash_16^3x32_nv12_fp32", "op": "wilson", "dims": list(dims), "nv": nv,
                   "m0": m0, "c_sw": 0, "links": "exp(0.3 i H), seed 1", "rhs": "CN(0,1), seed 101",
                   "flops_per_site_rhs": 1320, "bytes_per_site": site_bytes("wilson", nv, 8),
                   "rotating_sets": args.rotate},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rows": rows,
    }
    if copy_row:
        out["copy_calibration"] = copy_row
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
