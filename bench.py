"""Benchmark: DA-CSR (int16 offsets) vs CSR (int32 columns) SpMV on one MI355X.

One step = one DA-CSR SpMV y = A x (float64, beta = 0) on the 3D 27-point
stencil over a 128^3 grid in natural order (n 2,097,152, nnz 55,742,968,
bandwidth 16513).  `value` is the effective bandwidth of that step under the
traffic model of Eq. 3 plus x and y (Sec. 4):
    T = 4 (n+1) + nnz (2 + 8) + 8 n (x) + 8 n (y)
divided by the measured time per step.  The CSR comparison, the streaming
ceiling and the CPU oracle baseline are measured in the same run, outside the
timed steps, and reported beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def model_bytes(nrows, ncols, nnz, iindex, scalar=8, nrhs=1, beta_nonzero=False):
    # Eq. 3 with int32 row pointers, plus x read once and y written (and read)
    return (4 * (nrows + 1) + nnz * (iindex + scalar) + scalar * nrhs * ncols
            + scalar * nrhs * nrows * (2 if beta_nonzero else 1))


def time_launches(fn, reps):
    """Mean seconds per call of fn() over reps back-to-back calls (HIP events
    on torch's current stream, which is the stream the library launches on)."""
    import torch

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) * 1e-3 / reps


def epochs(fn, reps, n_epochs=5):
    """Minimum over epochs of the mean time per call (the paper's nanobench
    protocol takes the minimum over epochs)."""
    return min(time_launches(fn, reps) for _ in range(n_epochs))


def cpu_native(A, e, x, budget_s=3.0):
    """The native CPU baseline (C++ with OpenMP, rows split statically, four
    partial sums per row): DA-CSR and CSR SpMV on all host cores the process
    may use and on one thread, minimum over epochs of the mean time; the DA
    uplift beside the paper's CPU figures."""
    import numpy as np

    from paper_2307_06305_amd import cpu

    ncores = len(os.sched_getaffinity(0))
    da = cpu.arrays(e["rowptr"], e["off"], e["vals"], x, np.int16)
    cs = cpu.arrays(A.rowptr, A.colids, A.vals, x, np.int32)
    y = np.empty(A.nrows)
    T_da = model_bytes(A.nrows, A.ncols, A.nnz, 2)
    T_csr = model_bytes(A.nrows, A.ncols, A.nnz, 4)
    out = {"cores": ncores, "cpu": _cpu_model(), "kind": "native C++ OpenMP"}
    for threads in sorted({ncores, 1}, reverse=True):
        row = {}
        for name, fn, arrs, T in (("da", cpu.spmv_da, da, T_da), ("csr", cpu.spmv_csr, cs, T_csr)):
            fn(A.nrows, arrs[0], arrs[1], arrs[2], arrs[3], y, threads)  # warm
            t0 = time.perf_counter()
            fn(A.nrows, arrs[0], arrs[1], arrs[2], arrs[3], y, threads)
            once = time.perf_counter() - t0
            reps = max(1, int(budget_s / 5 / max(once, 1e-6)))
            best = None
            for _ in range(5):
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn(A.nrows, arrs[0], arrs[1], arrs[2], arrs[3], y, threads)
                dt = (time.perf_counter() - t0) / reps
                best = dt if best is None else min(best, dt)
            row[name] = {"ms": round(best * 1e3, 3), "gbs": round(T / best / 1e9, 2)}
        row["uplift"] = round(row["csr"]["ms"] / row["da"]["ms"] - 1.0, 4)
        out[f"threads_{threads}"] = row
        log(f"cpu native, {threads} threads: {row}")
    out["predicted_uplift"] = round(T_csr / T_da - 1.0, 4)
    out["paper_cpu_context"] = {"uplift_st": 0.11, "uplift_mt": 0.175, "predicted": 0.20}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, e, x, budget_s=12.0):
    """The CPU oracle's DA-CSR SpMV on the same matrix, repeated until about
    budget_s seconds have passed (NumPy, one thread)."""
    from oracle.spmv import spmv_da

    reps = 0
    t0 = time.perf_counter()
    while True:
        spmv_da(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], x)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    return dt, reps


def spmv_pair(D, M, Cm, n, ncols, nnz, xd, tune_reps):
    """Autotune and time a DA handle M and a CSR handle Cm on the same x."""
    import torch

    from paper_2307_06305_amd.tuning import autotune, config_name

    y = torch.zeros(n, dtype=torch.float64, device=xd.device)
    out = {}
    for name, mat, iidx in (("da", M, 2), ("csr", Cm, 4)):
        if mat is None:
            continue
        best, _ = autotune(mat, xd, y, reps=tune_reps)
        t = epochs(lambda: mat.apply(xd, y), 30)
        T = model_bytes(n, ncols, nnz, iidx)
        out[name] = {"us": round(t * 1e6, 2), "gbs": round(T / t / 1e9, 1),
                     "pct_hbm_peak": round(100 * T / t / 1e9 / HBM_PEAK_GBS, 2),
                     "launch": config_name(best)}
    if "da" in out and "csr" in out:
        out["speedup"] = round(out["csr"]["us"] / out["da"]["us"], 4)
        out["predicted_speedup"] = round(model_bytes(n, ncols, nnz, 4) / model_bytes(n, ncols, nnz, 2), 4)
    return out


def bench_banded(D, args):
    """Random banded n = 4M (lognormal rows, half-width 20000): DA vs CSR in
    natural order; the scrambled copy: CSR as scrambled, then host reordering
    (RCM + refinement) and DA vs CSR in the new order."""
    import numpy as np
    import torch

    from workloads import config_matrix, config_vector

    dev = torch.device("cuda:0")
    out = {}
    A = config_matrix(2)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    x = torch.from_numpy(config_vector(2, A.ncols)).to(dev)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    out["natural"] = {"n": A.nrows, "nnz": A.nnz, "bandwidth": e["w"],
                      **spmv_pair(D, M, Cm, A.nrows, A.ncols, A.nnz, x, args.tune_reps)}
    M.destroy()
    Cm.destroy()
    # the same number of scattered x reads without the matrix: the gather
    # rate the products cannot exceed (and, for context, narrower and wider
    # scatter)
    sink = torch.zeros(65536, dtype=torch.float64, device=dev)
    per_row = int(round(A.nnz / A.nrows))
    probe = {"rows": A.nrows, "per_row": per_row, "reads": A.nrows * per_row}
    for hw in (64, 20000, 2000000):
        fn = lambda: D.gather_read(x, sink, A.nrows, per_row, halfwidth=hw)
        t = epochs(fn, 20)
        probe[f"hw{hw}_us"] = round(t * 1e6, 1)
        probe[f"hw{hw}_greads_per_s"] = round(A.nrows * per_row / t / 1e9, 1)
    out["natural"]["gather_probe"] = probe
    del A, e
    log(f"banded natural: {out['natural']}")
    Q = config_matrix(2, scrambled=True)
    w_scr = D.fit_check(Q.nrows, Q.ncols, Q.rowptr, Q.colids)[0]
    Cq = D.Matrix.csr_create(Q.nrows, Q.ncols, Q.rowptr, Q.colids, Q.vals)
    scr = spmv_pair(D, None, Cq, Q.nrows, Q.ncols, Q.nnz, x, args.tune_reps)
    Cq.destroy()
    t0 = time.time()
    e = D.encode(Q.nrows, Q.ncols, Q.rowptr, Q.colids, Q.vals, allow_rcm=True)
    t_enc = time.time() - t0
    # the reordered matrix in CSR form too, for the iso-order comparison
    cols = (np.repeat(np.arange(Q.nrows, dtype=np.int64), np.diff(e["rowptr"]))
            + e["off"].astype(np.int64)).astype(np.int32)
    M = D.Matrix.create(Q.nrows, Q.ncols, e["rowptr"], e["off"], e["vals"])
    Cr = D.Matrix.csr_create(Q.nrows, Q.ncols, e["rowptr"], cols, e["vals"])
    out["scrambled"] = {"bandwidth_scrambled": w_scr, "bandwidth_reordered": e["w"],
                        "reorder_encode_s": round(t_enc, 2), "csr_scrambled_order": scr["csr"],
                        **spmv_pair(D, M, Cr, Q.nrows, Q.ncols, Q.nnz, x, args.tune_reps)}
    M.destroy()
    Cr.destroy()
    log(f"banded scrambled: {out['scrambled']}")
    return out


def bench_cg(D, args):
    """Time to 1e-10 relative residual: float64 CG against mixed-precision
    iterative refinement (float32 DA-CSR inner solves), 7-point Poisson on a
    128 x 128 x 1024 box (n 16,777,216), b uniform on [-1, 1], x0 = 0."""
    import torch

    from workloads import config_matrix, config_vector

    dev = torch.device("cuda:0")
    A = config_matrix(3)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    A64 = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], store=D.F64)
    A32 = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], store=D.F32)
    b = torch.from_numpy(config_vector(3, A.nrows)).to(dev)
    x64 = torch.zeros_like(b)
    xm = torch.zeros_like(b)
    from paper_2307_06305_amd.tuning import STREAM, autotune, candidates, config_name
    stream_cfgs = [c for c in candidates() if c[0] == STREAM and c[1] <= 16]
    best64, _ = autotune(A64, b, x64, configs=stream_cfgs, reps=args.tune_reps)
    b32 = b.float()
    y32 = torch.zeros_like(b32)
    best32, _ = autotune(A32, b32, y32, configs=stream_cfgs, reps=args.tune_reps)
    del b32, y32
    res = {"workload": "poisson3d_7pt_128x128x1024", "n": A.nrows, "nnz": A.nnz,
           "bandwidth": e["w"], "tol": 1e-10, "launch_f64": config_name(best64),
           "launch_f32": config_name(best32)}
    for name, a32, xv in (("fp64", None, x64), ("mixed", A32, xm)):
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = D.cg(A64, b, xv, A32=a32, tol=1e-10, inner_tol=1e-5, max_iter=20000,
                        check_every=32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        res[name] = {"s": round(best, 4), **info}
        log(f"cg {name}: {res[name]}")
    res["speedup_mixed"] = round(res["fp64"]["s"] / res["mixed"]["s"], 3)
    res["mixed_vs_fp64_rel_err"] = float(((xm - x64).norm() / x64.norm()).item())
    A64.destroy()
    A32.destroy()
    return res


SWEEP_N = (16, 24, 32, 48, 64, 80, 96, 112, 128, 160)


def graph_time(fn, min_s=0.05, n_epochs=7):
    """Minimum over epochs of the time per call, with K back-to-back calls of
    fn captured in one HIP graph (K sized so an epoch lasts about min_s), so
    that small products are not timed through the Python call overhead."""
    import torch

    fn()
    t1 = time_launches(fn, 5)
    k = max(10, min(2000, int(min_s / max(t1, 1e-7))))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(k):
            fn()
    g.replay()
    torch.cuda.synchronize()
    best = min(time_launches(g.replay, 1) for _ in range(n_epochs)) / k
    del g
    return best, k


def graph_autotune(mat, x, y):
    """The autotuner for products of a few microseconds: every candidate
    configuration timed through captured graphs; sets and returns the fastest."""
    from paper_2307_06305_amd.tuning import candidates_for

    times = {}
    for c in candidates_for(mat):
        mat.set_config(*c)
        times[c] = graph_time(lambda: mat.apply(x, y), min_s=0.004, n_epochs=3)[0]
    best = min(times, key=times.get)
    mat.set_config(*best)
    return best


def bench_sweep(D, args):
    """DA-CSR against CSR on the 27-point stencil over N^3 grids from 16 to
    160: relative speed and throughput against the working-set size, with
    the L2 (4 MB per XCD, 32 MB in all) and MALL (256 MB) boundaries.  No
    cache flush between products: a set that fits a cache level stays there,
    as in the paper's Fig. 4."""
    import torch

    from paper_2307_06305_amd.tuning import autotune, config_name
    from workloads.matrices import stencil_3d_27pt, uniform_vector

    dev = torch.device("cuda:0")
    rows = []
    for N in SWEEP_N:
        A = stencil_3d_27pt(N, 1001)
        e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
        M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
        Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
        x = torch.from_numpy(uniform_vector(A.ncols, 2001)).to(dev)
        y = torch.zeros(A.nrows, dtype=torch.float64, device=dev)
        T_da = model_bytes(A.nrows, A.ncols, A.nnz, 2)
        T_csr = model_bytes(A.nrows, A.ncols, A.nnz, 4)
        row = {"N": N, "n": A.nrows, "nnz": A.nnz, "bandwidth": e["w"],
               "csr_mb": round(T_csr / 1e6, 2),
               "regime": "L2" if T_csr <= 32e6 else ("MALL" if T_csr <= 256e6 else "HBM")}
        for name, mat, T in (("da", M, T_da), ("csr", Cm, T_csr)):
            mat.apply(x, y)
            if time_launches(lambda: mat.apply(x, y), 5) < 50e-6:
                best = graph_autotune(mat, x, y)
            else:
                best, _ = autotune(mat, x, y, reps=max(3, args.tune_reps // 2))
            t, k = graph_time(lambda: mat.apply(x, y))
            row[name] = {"us": round(t * 1e6, 3), "gbs": round(T / t / 1e9, 1),
                         "launch": config_name(best), "graph_launches": k}
            if best[0] == D.VAR_STREAM:
                # the same launch with the matrix loaded plainly (kept in
                # the MALL when the working set fits it)
                mat.set_config(*best, cache=D.CACHE_PLAIN)
                tp, _ = graph_time(lambda: mat.apply(x, y))
                mat.set_config(*best)
                row[name]["us_plain"] = round(tp * 1e6, 3)
                row[name]["gbs_plain"] = round(T / tp / 1e9, 1)
        row["speedup"] = round(row["csr"]["us"] / row["da"]["us"], 4)
        row["predicted_speedup"] = round(T_csr / T_da, 4)
        log(f"sweep N={N}: {row}")
        rows.append(row)
        M.destroy()
        Cm.destroy()
        del A, e
    return rows


MALL_MB = (4, 16, 32, 64, 96, 128, 192, 256, 384, 512, 1024, 2048)


def bench_mall(D, args):
    """Read ceilings by working-set size: a buffer of S MB read over and over
    (no flush), along each read path of the probe (16-byte loads into
    registers or direct-to-LDS tiles of 8 KiB, the 27-point product's tile
    size; non-temporal or plain).  A buffer that fits a cache level is
    served from it on repeated reads: L2 is 4 MB per XCD (32 MB in all, each
    XCD reading its own eighth), the MALL 256 MB.  Two timings per path:
    one pass per launch, back to back (`<path>_gbs`, the regime of the
    product sweep), and about 1 GiB per launch as repeated passes over the
    buffer (`<path>_multi_gbs`), which pays the launch's ramp-up once and so
    shows the rate of the level that serves the re-reads."""
    import torch

    dev = torch.device("cuda:0")
    sink = torch.zeros(65536, dtype=torch.float64, device=dev)
    modes = (("nt", D.READ_NT), ("plain", D.READ_PLAIN), ("lds_nt", D.READ_LDS_NT),
             ("lds_plain", D.READ_LDS_PLAIN))
    rows = []
    for mb in MALL_MB:
        buf = torch.empty(mb << 20, dtype=torch.uint8, device=dev)
        buf.fill_(1)
        passes = max(1, 1024 // mb)
        row = {"mb": mb, "passes": passes}
        for name, mode in modes:
            fn = lambda: D.stream_read(buf, sink, mode, 8192)
            fn()
            t1 = time_launches(fn, 3)
            reps = max(5, min(2000, int(0.02 / max(t1, 1e-7))))
            t = min(time_launches(fn, reps) for _ in range(3))
            row[f"{name}_gbs"] = round(buf.numel() / t / 1e9, 1)
            fm = lambda: D.stream_read(buf, sink, mode, 8192, passes=passes)
            fm()
            tm = min(time_launches(fm, 10) for _ in range(3))
            row[f"{name}_multi_gbs"] = round(passes * buf.numel() / tm / 1e9, 1)
        log(f"mall probe {mb} MB: {row}")
        rows.append(row)
        del buf
    return {"tile_bytes": 8192, "read": rows}


def bench_cg_cube(D, args):
    """The 7-point Poisson operator on the 256^3 cube (n 16,777,216): its
    bandwidth, 65536 in natural order, stays above the 16-bit range after RCM,
    so the solve runs on int32 CSR, float64 CG against mixed precision with
    float32-valued CSR inner solves."""
    import torch

    from paper_2307_06305_amd.tuning import STREAM, autotune, candidates, config_name
    from workloads import config_vector
    from workloads.matrices import poisson_3d_7pt

    dev = torch.device("cuda:0")
    A = poisson_3d_7pt(256, 256, 256)
    w, _, _, fits = D.fit_check(A.nrows, A.ncols, A.rowptr, A.colids)
    t0 = time.time()
    perm = D.rcm(A.nrows, A.rowptr, A.colids)
    _, w_rcm, fits_rcm = D.refine_bandwidth(A.nrows, A.rowptr, A.colids, perm, max_sweeps=0)
    t_rcm = time.time() - t0
    del perm
    C64 = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, store=D.F64)
    C32 = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, store=D.F32)
    b = torch.from_numpy(config_vector(3, A.nrows)).to(dev)
    x64 = torch.zeros_like(b)
    xm = torch.zeros_like(b)
    stream_cfgs = [c for c in candidates() if c[0] == STREAM and c[1] <= 16]
    best64, _ = autotune(C64, b, x64, configs=stream_cfgs, reps=args.tune_reps)
    b32 = b.float()
    y32 = torch.zeros_like(b32)
    best32, _ = autotune(C32, b32, y32, configs=stream_cfgs, reps=args.tune_reps)
    del b32, y32
    res = {"workload": "poisson3d_7pt_256^3", "n": A.nrows, "nnz": A.nnz,
           "bandwidth": w, "fits_int16": bool(fits), "bandwidth_rcm": w_rcm,
           "fits_int16_rcm": bool(fits_rcm), "rcm_s": round(t_rcm, 2), "index": "int32 CSR",
           "tol": 1e-10, "launch_f64": config_name(best64), "launch_f32": config_name(best32)}
    for name, a32, xv in (("fp64", None, x64), ("mixed", C32, xm)):
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = D.cg(C64, b, xv, A32=a32, tol=1e-10, inner_tol=1e-5, max_iter=20000,
                        check_every=32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        res[name] = {"s": round(best, 4), **info}
        log(f"cg cube {name}: {res[name]}")
    res["speedup_mixed"] = round(res["fp64"]["s"] / res["mixed"]["s"], 3)
    res["mixed_vs_fp64_rel_err"] = float(((xm - x64).norm() / x64.norm()).item())
    C64.destroy()
    C32.destroy()
    return res


def _grid_cell(D, A, fmt, store, x64, tune_reps, graph=False):
    """Upload A in one storage cell, tune it, time it; model bytes with the
    cell's index and scalar sizes (x and y float32 unless float64 values)."""
    import numpy as np
    import torch

    from paper_2307_06305_amd.tuning import autotune, config_name

    idx, _ = D.encode_index(fmt, A.nrows, A.ncols, A.rowptr, A.colids)
    M = D.Matrix.create_format(fmt, A.nrows, A.ncols, A.rowptr, idx, A.vals, store=store)
    del idx
    f64 = store == D.F64
    x = torch.from_numpy(x64 if f64 else x64.astype(np.float32)).to("cuda")
    y = torch.zeros(A.nrows, dtype=torch.float64 if f64 else torch.float32, device="cuda")
    M.apply(x, y)
    if graph:
        best = graph_autotune(M, x, y)
        t = graph_time(lambda: M.apply(x, y))[0]
    else:
        best, _ = autotune(M, x, y, reps=tune_reps)
        t = epochs(lambda: M.apply(x, y), 30)
    ib = np.dtype(D.FORMATS[fmt][0]).itemsize
    sb = np.dtype(D.VALUE_DTYPES[store]).itemsize
    T = model_bytes(A.nrows, A.ncols, A.nnz, ib, scalar=sb)
    if store == D.F16:  # x and y are float32: 4 bytes per element, not 2
        T += 2 * (A.ncols + A.nrows)
    M.destroy()
    return {"us": round(t * 1e6, 3), "model_bytes": T, "gbs": round(T / t / 1e9, 1),
            "launch": config_name(best)}


def bench_grid(D, args):
    """The storage grid of Fig. 3 on the GPU: index widths (int8 / int16 DA
    offsets, int32 / int16 CSR columns) against scalar widths (float64 /
    float32 / float16), with the model's predicted speedups; the non-square
    products of the remark in Sec. 4."""
    import numpy as np

    from workloads import config_matrix, config_vector, stencil_3d_27pt
    from workloads.matrices import random_banded, stencil_3d_27pt_box, uniform_vector

    names = {D.FORMAT_DA16: "da16", D.FORMAT_CSR32: "csr32", D.FORMAT_DA8: "da8",
             D.FORMAT_CSR16: "csr16"}
    vnames = {D.F64: "f64", D.F32: "f32", D.F16: "f16"}
    out = {}

    def table(A, x, fmts, graph=False):
        cells = {}
        for fmt in fmts:
            for st in (D.F64, D.F32, D.F16):
                c = _grid_cell(D, A, fmt, st, x, args.tune_reps, graph)
                cells[f"{names[fmt]}_{vnames[st]}"] = c
                log(f"grid {A.name} {names[fmt]} {vnames[st]}: {c}")
        base = cells[f"{names[fmts[0]]}_f64"]
        for c in cells.values():
            c["speedup"] = round(base["us"] / c["us"], 4)
            c["predicted_speedup"] = round(base["model_bytes"] / c["model_bytes"], 4)
        return cells

    # 27-point stencil on a 10 x 10 x 20972 box: w = 111 fits int8 offsets
    A = stencil_3d_27pt_box(10, 10, 20972, 1009)
    x = uniform_vector(A.ncols, 2009)
    out["box_10x10x20972"] = {"n": A.nrows, "nnz": A.nnz, "bandwidth": 111,
                              "cells": table(A, x, [D.FORMAT_CSR32, D.FORMAT_DA16, D.FORMAT_DA8])}
    del A
    # the 128^3 stencil: DA16 against CSR32 with each scalar type (the
    # multi-precision remark after Fig. 3: f64 -> f32 gains 3/2 for CSR32 and
    # 5/3 for DA16 in the matrix traffic)
    A = config_matrix(1)
    x = config_vector(1, A.ncols)
    cells = table(A, x, [D.FORMAT_CSR32, D.FORMAT_DA16])
    out["stencil_128^3"] = {"n": A.nrows, "nnz": A.nnz, "cells": cells,
                            "f64_to_f32": {"csr32": round(cells["csr32_f64"]["us"] / cells["csr32_f32"]["us"], 4),
                                           "da16": round(cells["da16_f64"]["us"] / cells["da16_f32"]["us"], 4)}}
    del A
    # same index width: DA16 against CSR16 (remark closing Sec. 4), on the
    # largest 27-point cube whose columns fit int16 (32^3 = 32768 rows; its
    # products sit in L2 and are timed through captured graphs)
    A = stencil_3d_27pt(32, 1001)
    x = uniform_vector(A.ncols, 2001)
    cells = {}
    for fmt in (D.FORMAT_CSR16, D.FORMAT_DA16):
        c = _grid_cell(D, A, fmt, D.F64, x, args.tune_reps, graph=True)
        cells[names[fmt] + "_f64"] = c
    cells["da16_over_csr16"] = round(cells["csr16_f64"]["us"] / cells["da16_f64"]["us"], 4)
    out["same_index_width_27pt_32^3"] = cells
    log(f"grid same index width: {cells}")
    # non-square (Sec. 4 remark): wide and tall random bands, n = 4M
    for name, nr, nc in (("wide", 4_000_000, 4_040_000), ("tall", 4_040_000, 4_000_000)):
        A = random_banded(nr, 1012, half_band=20000, ncols=nc)
        x = uniform_vector(A.ncols, 2012)
        res = {"nrows": nr, "ncols": nc, "nnz": A.nnz}
        for fmt in (D.FORMAT_CSR32, D.FORMAT_DA16):
            res[names[fmt]] = _grid_cell(D, A, fmt, D.F64, x, args.tune_reps)
        res["speedup"] = round(res["csr32"]["us"] / res["da16"]["us"], 4)
        res["predicted_speedup"] = round(res["csr32"]["model_bytes"] / res["da16"]["model_bytes"], 4)
        out[name] = res
        log(f"grid {name}: {res}")
        del A
    return out


def bsr_model_bytes(nbrows, nbcols, nnzb, b, iindex, scalar=8):
    # Eq. 3 with one index per block and b*b scalars per block, plus x and y
    return 4 * (nbrows + 1) + nnzb * (iindex + b * b * scalar) + scalar * b * (nbcols + nbrows)


def bench_blocks(D, args):
    """DA-BSR against BSR (Sec. 1: diagonal addressing applied to block
    storage) on a block matrix of the finite-element kind: 3 x 3 blocks on
    the 27-point pattern of a 64^3 node grid (786,432 rows, 6.86M blocks),
    float64 and float32; the same matrix in scalar DA-CSR and CSR."""
    import torch

    from paper_2307_06305_amd.tuning import autotune, config_name
    from workloads.matrices import block_stencil_27pt, uniform_vector

    b = 3
    A = block_stencil_27pt(64, b, 1010)
    x64 = uniform_vector(A.ncols, 2010)
    nbr = A.nrows // b
    out = {"workload": "block3_stencil27_64^3", "rows": A.nrows, "nnz": A.nnz, "block": b}
    for fmt, name, ib in ((D.FORMAT_BSR32, "bsr32", 4), (D.FORMAT_DABSR16, "dabsr16", 2)):
        e = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b, fmt)
        nnzb = len(e["bidx"])
        out["nnzb"] = nnzb
        out["block_bandwidth"] = e["wb"]
        for store, sname, sb in ((D.F64, "f64", 8), (D.F32, "f32", 4)):
            M = D.Matrix.bsr_create(fmt, nbr, nbr, b, e["browptr"], e["bidx"], e["bvals"],
                                    store=store)
            tdt = torch.float64 if store == D.F64 else torch.float32
            x = torch.from_numpy(x64).to("cuda", tdt)
            y = torch.zeros(A.nrows, dtype=tdt, device="cuda")
            best, _ = autotune(M, x, y, reps=args.tune_reps)
            t = epochs(lambda: M.apply(x, y), 30)
            T = bsr_model_bytes(nbr, nbr, nnzb, b, ib, sb)
            out[f"{name}_{sname}"] = {"us": round(t * 1e6, 2), "model_bytes": T,
                                      "gbs": round(T / t / 1e9, 1), "launch": config_name(best)}
            log(f"blocks {name} {sname}: {out[f'{name}_{sname}']}")
            M.destroy()
        del e
    for fmt, name in ((D.FORMAT_CSR32, "csr32"), (D.FORMAT_DA16, "da16")):
        c = _grid_cell(D, A, fmt, D.F64, x64, args.tune_reps)
        out[f"{name}_f64"] = c
        log(f"blocks scalar {name}: {c}")
    for s in ("f64", "f32"):
        out[f"speedup_dabsr_over_bsr_{s}"] = round(
            out[f"bsr32_{s}"]["us"] / out[f"dabsr16_{s}"]["us"], 4)
        out[f"predicted_{s}"] = round(
            out[f"bsr32_{s}"]["model_bytes"] / out[f"dabsr16_{s}"]["model_bytes"], 4)
    out["speedup_dabsr_over_csr32_f64"] = round(out["csr32_f64"]["us"] / out["dabsr16_f64"]["us"], 4)
    return out


def bench_spmm(D, args):
    """SpMM Y = A X with nrhs = 1, 2, 4, 8 interleaved right-hand sides on the
    27-point 128^3 matrix, DA-CSR and CSR: each index and value is read
    once for all right-hand sides."""
    import numpy as np
    import torch

    from workloads import config_matrix

    A = config_matrix(1)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    g = torch.Generator().manual_seed(2101)
    out = {"workload": "stencil3d_27pt_128^3"}
    for k in (1, 2, 4, 8):
        X = (torch.rand(A.ncols, k, generator=g, dtype=torch.float64) * 2 - 1).to("cuda")
        Y = torch.zeros(A.nrows, k, dtype=torch.float64, device="cuda")
        row = {}
        for name, mat, ib in (("da", M, 2), ("csr", Cm, 4)):
            T = model_bytes(A.nrows, A.ncols, A.nnz, ib, nrhs=k)
            row[name] = {"model_bytes": T}
            for vname, variant in (("stream", D.VAR_STREAM), ("vector", D.VAR_VECTOR)):
                t_best = None
                tiles = (1024, 2048) if variant == D.VAR_STREAM else (2048,)
                for lanes in (1, 2, 4, 8, 16):
                    for tile in tiles:
                        mat.set_config(variant, lanes, 1, tile)
                        mat.spmm(X, Y)
                        t = epochs(lambda: mat.spmm(X, Y), 10, 3)
                        if t_best is None or t < t_best[0]:
                            t_best = (t, lanes, tile)
                row[name][vname] = {"us": round(t_best[0] * 1e6, 1), "lanes": t_best[1],
                                    "gbs": round(T / t_best[0] / 1e9, 1)}
                if variant == D.VAR_STREAM:
                    row[name][vname]["tile"] = t_best[2]
            best = min(row[name]["stream"]["us"], row[name]["vector"]["us"])
            row[name]["us"] = best
            row[name]["gbs"] = round(T / (best * 1e-6) / 1e9, 1)
        row["speedup"] = round(row["csr"]["us"] / row["da"]["us"], 4)
        out[f"nrhs{k}"] = row
        log(f"spmm nrhs={k}: {row}")
    M.destroy()
    Cm.destroy()
    return out


def bench_coo(D, args):
    """DA-COO against COO (Sec. 1: diagonal addressing applied to one index
    vector of COO) on the 27-point 128^3 matrix; both stream a 4-byte row
    index per entry on top of DA-CSR / CSR."""
    import torch

    from workloads import config_matrix, config_vector

    A = config_matrix(1)
    x = torch.from_numpy(config_vector(1, A.ncols)).to("cuda")
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    out = {"workload": "stencil3d_27pt_128^3", "n": A.nrows, "nnz": A.nnz}
    for fmt, name, ib in ((D.FORMAT_COO32, "coo32", 4), (D.FORMAT_DACOO16, "dacoo16", 2)):
        rows, idx = D.coo_encode(A.nrows, A.ncols, A.rowptr, A.colids, fmt)
        M = D.Matrix.coo_create(fmt, A.nrows, A.ncols, rows, idx, A.vals)
        del rows, idx
        M.apply(x, y)
        t = epochs(lambda: M.apply(x, y), 30)
        T = A.nnz * (4 + ib + 8) + 8 * A.ncols + 8 * A.nrows
        out[name] = {"us": round(t * 1e6, 2), "model_bytes": T, "gbs": round(T / t / 1e9, 1)}
        log(f"coo {name}: {out[name]}")
        M.destroy()
    out["speedup"] = round(out["coo32"]["us"] / out["dacoo16"]["us"], 4)
    out["predicted_speedup"] = round(out["coo32"]["model_bytes"] / out["dacoo16"]["model_bytes"], 4)
    return out


def bench_batch(D, args):
    """512 DA-CSR matrices (n log-uniform on [1e3, 2e5]; 2D 5-point, 3D
    7-point, 3D 27-point and random banded; 1-8 right-hand sides): one
    persistent graph-captured launch against 512 separately tuned launches."""
    import numpy as np
    import torch

    from workloads.matrices import batch_matrix, batch_member

    dev = torch.device("cuda:0")
    count = args.batch_count
    mats, Xs, Ys, shapes = [], [], [], []
    total_nnz = total_rows = 0
    t0 = time.time()
    for i in range(count):
        d = batch_member(1004, i)
        A = batch_matrix(d)
        e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
        M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
        k = d["nrhs"]
        g = torch.Generator(device="cpu").manual_seed(7000 + i)
        Xs.append((torch.rand(A.ncols, k, generator=g, dtype=torch.float64) * 2 - 1).to(dev))
        Ys.append(torch.zeros(A.nrows, k, dtype=torch.float64, device=dev))
        mats.append(M)
        shapes.append((D.features(A.nrows, A.ncols, A.rowptr, A.colids, 1),
                       D.features(A.nrows, A.ncols, A.rowptr, A.colids, k)))
        total_nnz += A.nnz
        total_rows += A.nrows
    log(f"batch: {count} matrices, {total_rows} rows, {total_nnz} entries "
        f"({time.time() - t0:.1f}s to build)")
    # separate launches: the native autotuner picks each matrix's SpMV and
    # SpMM configuration (the SpMM one stays set); its timings also score the
    # shipped selector network against the exhaustive search
    from paper_2307_06305_amd import selector as S

    feats, times, default = [], [], []
    sum_best = 0.0

    def tuned_times(M, k, X, Y):
        # three autotuner runs, averaged: the selector's regret divides by the
        # fastest of 63 timings, a minimum that one noisy run biases low (the
        # last run leaves its own fastest class set)
        return np.mean([D.autotune(M, k, X, Y, reps=3) for _ in range(3)], axis=0)

    for M, X, Y, A_shape in zip(mats, Xs, Ys, shapes):
        default_cfg = M.get_config()
        k = X.shape[1]
        x1 = X[:, 0].contiguous()
        y1 = torch.zeros(M.nrows, dtype=torch.float64, device=dev)
        times.append(tuned_times(M, 1, x1, y1))
        feats.append(A_shape[0])
        default.append(S.config_class(default_cfg, 1))
        if k > 1:
            times.append(tuned_times(M, k, X, Y))
            feats.append(A_shape[1])
            default.append(S.config_class(default_cfg, k))
        sum_best += float(np.min(times[-1]))  # this matrix's own product, best class
    sel = S.evaluate(S.load_weights(), np.array(feats), np.array(times), np.array(default))
    sel["with_autotuner_fallback"] = [
        S.evaluate_fallback(S.load_weights(), np.array(feats), np.array(times), th)
        for th in (0.1, 0.2, 0.3, 0.5)]
    log(f"selector on the batch matrices: {sel}")

    def separate():
        for M, X, Y in zip(mats, Xs, Ys):
            if X.shape[1] == 1:
                M.apply(X.view(-1), Y.view(-1))
            else:
                M.spmm(X, Y)

    t_sep = epochs(separate, 3, 3)
    # one launch; each matrix reduces its rows with the lane count of its
    # stream configuration: first the default for its mean row length, then
    # the one the autotuner picked for its own product above
    t_graph_by = {}
    for how in ("default_lanes", "tuned_lanes"):
        if how == "default_lanes":
            tuned = [M.get_config() for M in mats]
            for M in mats:
                mean = M.nnz / max(M.nrows, 1)
                g = 1 if mean < 4 else 2
                while g < 16 and g * 16 < mean:
                    g *= 2
                M.set_config(D.VAR_STREAM, g, 1, 2048)
        else:
            for M, c in zip(mats, tuned):
                M.set_config(D.VAR_STREAM, c["lanes"], 1, 2048)
        Bt = D.Batch(mats, Xs, Ys, 1.0, 0.0, workgroups=args.batch_workgroups)
        t_graph_by[how] = epochs(lambda: Bt.run(use_graph=True), 10, 5)
        Bt.destroy()
    log(f"batch graph by lane choice: {t_graph_by}")
    best_how = min(t_graph_by, key=t_graph_by.get)
    if best_how == "default_lanes":
        for M in mats:
            mean = M.nnz / max(M.nrows, 1)
            g = 1 if mean < 4 else 2
            while g < 16 and g * 16 < mean:
                g *= 2
            M.set_config(D.VAR_STREAM, g, 1, 2048)
    B = D.Batch(mats, Xs, Ys, 1.0, 0.0, workgroups=args.batch_workgroups)
    info = B.info()
    t_graph = epochs(lambda: B.run(use_graph=True), 10, 5)
    t_direct = epochs(lambda: B.run(use_graph=False), 10, 5)
    # the persistent grid (1024 workgroups walking equal-work ranges), for comparison
    Bp = D.Batch(mats, Xs, Ys, 1.0, 0.0, workgroups=1024)
    t_persist = epochs(lambda: Bp.run(use_graph=True), 10, 5)
    Bp.destroy()
    T = info["model_bytes"]
    res = {"matrices": count, "rows": total_rows, "nnz": total_nnz, "tiles": info["ntiles"],
           "workgroups": info["workgroups"], "model_bytes": T,
           "graph_us": round(t_graph * 1e6, 1), "graph_gbs": round(T / t_graph / 1e9, 1),
           "lanes": best_how,
           "graph_us_by_lanes": {k: round(v * 1e6, 1) for k, v in t_graph_by.items()},
           "direct_us": round(t_direct * 1e6, 1),
           "persistent_1024_us": round(t_persist * 1e6, 1),
           "separate_us": round(t_sep * 1e6, 1), "separate_gbs": round(T / t_sep / 1e9, 1),
           "sum_of_tuned_kernel_us": round(sum_best * 1e6, 1),
           "speedup_vs_separate": round(t_sep / t_graph, 3),
           "selector": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sel.items()}}
    res["selector"]["with_autotuner_fallback"] = [
        {k: round(v, 4) for k, v in fb.items()} for fb in sel["with_autotuner_fallback"]]
    log(f"batch: {res}")
    B.destroy()
    for M in mats:
        M.destroy()
    return res


def bench_selector_training(D, args):
    """Train a fresh selector network on the shipped autotuner dataset with
    the library's GPU training kernels; score it on the held-out matrices."""
    import numpy as np

    from paper_2307_06305_amd import selector as S

    d = np.load(S.DATASET, allow_pickle=False)
    data = {k: d[k] for k in d.files}
    tr, ho = S.split(data)
    t0 = time.time()
    params, losses = S.train(data["F"][tr], data["T"][tr], epochs=300, seed=11)
    dt = time.time() - t0
    ev = S.evaluate(params, data["F"][ho], data["T"][ho], data["default"][ho])
    res = {"train_samples": int(tr.sum()), "heldout_samples": int(ho.sum()), "train_s": round(dt, 2),
           "loss_first": round(float(losses[0]), 4), "loss_last": round(float(losses[-1]), 4),
           **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in ev.items()}}
    log(f"selector training: {res}")
    return res


def summary(res):
    """A compact digest of every figure the run measured, printed last on
    stderr (after the JSON line) so that a log cut to its tail still carries
    them; the headline comes last."""
    out = []

    def g(d, *keys):
        for k in keys:
            if not isinstance(d, dict) or k not in d:
                return None
            d = d[k]
        return d

    cb, cn = res.get("cpu_baseline"), res.get("cpu_native")
    if cb or cn:
        out.append(f"cpu: oracle {g(cb, 'value')}GB/s on 1 core | native DA/CSR uplift "
                   f"{g(cn, 'threads_16', 'uplift')} on {g(cn, 'cores')} threads, "
                   f"{g(cn, 'threads_1', 'uplift')} on 1")
    sp = res.get("spmm")
    if isinstance(sp, dict):
        parts = [f"{k[4:]}: {g(v, 'da', 'us')}/{g(v, 'csr', 'us')}us" for k, v in sp.items()
                 if k.startswith("nrhs") and isinstance(v, dict)]
        if parts:
            out.append("spmm DA/CSR " + ", ".join(parts))
    co, bl = res.get("coo"), res.get("blocks")
    if co or bl:
        out.append(f"dacoo/coo {g(co, 'dacoo16', 'us')}/{g(co, 'coo32', 'us')}us "
                   f"({g(co, 'speedup')}, model {g(co, 'predicted_speedup')}) | dabsr/bsr f64 "
                   f"{g(bl, 'dabsr16_f64', 'us')}/{g(bl, 'bsr32_f64', 'us')}us, f32 "
                   f"{g(bl, 'dabsr16_f32', 'us')}/{g(bl, 'bsr32_f32', 'us')}us")
    gr = res.get("grid")
    if isinstance(gr, dict):
        for wl, v in gr.items():
            if isinstance(v, dict) and "cells" in v:
                out.append(f"grid {wl} speedup over csr32_f64: " + ", ".join(
                    f"{c} {x.get('speedup')}" for c, x in v["cells"].items() if c != "csr32_f64"))
        sw_, wd, tl = gr.get("same_index_width_27pt_32^3"), gr.get("wide"), gr.get("tall")
        out.append(f"grid da16/csr16 {g(sw_, 'da16_over_csr16')} | wide DA/CSR "
                   f"{g(wd, 'speedup')} | tall {g(tl, 'speedup')}")
    sw = res.get("sweep")
    if sw:
        out.append("sweep N DA/CSR us (speedup) [plain DA]: " + ", ".join(
            f"{r['N']} {r['da']['us']}/{r['csr']['us']} ({r['speedup']}) "
            f"[{r['da'].get('us_plain')}]" for r in sw))
    if "mall" in res:
        rows = {r["mb"]: r for r in res["mall"].get("read", [])}
        out.append("read probe GB/s, 1 pass/launch | ~1 GiB of passes/launch (lds_nt, lds_plain): "
                   + ", ".join(f"{mb}MB {rows[mb]['lds_nt_gbs']}/{rows[mb]['lds_plain_gbs']} | "
                               f"{rows[mb].get('lds_nt_multi_gbs')}/"
                               f"{rows[mb].get('lds_plain_multi_gbs')}"
                               for mb in (64, 128, 256, 2048) if mb in rows))
    bt = res.get("batch")
    if bt:
        sel = bt.get("selector", {})
        out.append(f"batch512 graph {bt.get('graph_us')}us {bt.get('graph_gbs')}GB/s vs separate "
                   f"{bt.get('separate_us')}us | selector regret mean {sel.get('mean_regret')} "
                   f"p95 {sel.get('p95_regret')} within5% {sel.get('within_5pct')}")
    b = res.get("banded")
    if b:
        n, s = b.get("natural", {}), b.get("scrambled", {})
        gp = n.get("gather_probe", {})
        out.append(f"band4M DA {g(n, 'da', 'us')}us ({g(n, 'da', 'pct_hbm_peak')}%) CSR "
                   f"{g(n, 'csr', 'us')}us speedup {n.get('speedup')} (model "
                   f"{n.get('predicted_speedup')}) | gathers alone {gp.get('hw20000_us')}us | "
                   f"scrambled CSR {g(s, 'csr_scrambled_order', 'us')}us -> w "
                   f"{s.get('bandwidth_reordered')} DA {g(s, 'da', 'us')}us CSR "
                   f"{g(s, 'csr', 'us')}us")
    for key, name in (("cg_cube", "CG cube 256^3 CSR32"), ("cg", "CG box 128x128x1024 DA16")):
        c = res.get(key)
        if c:
            out.append(f"{name}: fp64 {g(c, 'fp64', 's')}s {g(c, 'fp64', 'iters')}it | mixed "
                       f"{g(c, 'mixed', 's')}s {g(c, 'mixed', 'outer')}x"
                       f"{g(c, 'mixed', 'iters')}it | speedup {c.get('speedup_mixed')}")
    da, csr = res.get("da", {}), res.get("csr", {})
    out.append(f"27pt128 DA {da.get('us')}us {da.get('gbs')}GB/s {da.get('pct_hbm_peak')}%peak | "
               f"CSR {csr.get('us')}us | speedup {res.get('speedup')} (model "
               f"{res.get('predicted_speedup')}, uplift frac {res.get('uplift_fraction')}) | "
               f"events {g(res, 'roofline', 'achieved')}GB/s frac {g(res, 'roofline', 'frac')} | "
               f"read ceiling {res.get('stream_read_gbs')}GB/s | gathers alone "
               f"{res.get('gather_probe_us')}us, stream at ceiling + gathers "
               f"{res.get('bound_us')}us")
    for line in out:
        print(f"[summary] {line}", file=sys.stderr, flush=True)


def profile_run(D, args):
    """A short run for rocprofv3: the copy probe of known size (the counters'
    calibration), then --profile-reps DA-CSR and CSR products of the chosen
    workload at fixed launch shapes, so each kernel symbol holds only these
    launches."""
    import numpy as np
    import torch

    from paper_2307_06305_amd.profiling import stream_launch
    from workloads import config_matrix, config_vector
    from workloads.matrices import stencil_3d_27pt, uniform_vector

    dev = torch.device("cuda:0")
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        D.stream_copy(src, dst)
    del src, dst
    wl = args.profile_workload
    if wl.startswith("read"):
        mb = int(wl[4:])
        buf = torch.empty(mb << 20, dtype=torch.uint8, device=dev)
        buf.fill_(1)
        sink = torch.zeros(65536, dtype=torch.float64, device=dev)
        passes = max(1, 1024 // mb)
        for mode in (D.READ_NT, D.READ_PLAIN, D.READ_LDS_NT, D.READ_LDS_PLAIN):
            for _ in range(20):
                D.stream_read(buf, sink, mode, 8192)
            for _ in range(5):
                D.stream_read(buf, sink, mode, 8192, passes=passes)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "done", "workload": wl, "copy_bytes": 1 << 30,
                          "read_bytes": mb << 20, "passes": passes}), flush=True)
        return
    if wl == "27pt":
        A, x = config_matrix(1), config_vector(1, 2097152)
    elif wl in ("band", "band_rcm"):
        A = config_matrix(2, scrambled=wl == "band_rcm")
        x = config_vector(2, A.ncols)
    elif wl.startswith("sweep"):
        A = stencil_3d_27pt(int(wl[5:]), 1001)
        x = uniform_vector(A.ncols, 2001)
    else:
        raise SystemExit(f"unknown --profile-workload {wl!r}")
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=wl == "band_rcm")
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    if e["permuted"]:
        cols = (np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(e["rowptr"]))
                + e["off"].astype(np.int64)).astype(np.int32)
        Cm = D.Matrix.csr_create(A.nrows, A.ncols, e["rowptr"], cols, e["vals"])
    else:
        Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    cache = D.CACHE_PLAIN if args.profile_cache == "plain" else D.CACHE_NT
    g, t, u = stream_launch(args.profile_da)
    M.set_config(D.VAR_STREAM, g, u, t, cache=cache)
    g, t, u = stream_launch(args.profile_csr)
    Cm.set_config(D.VAR_STREAM, g, u, t, cache=cache)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.zeros(A.nrows, dtype=torch.float64, device=dev)
    for _ in range(args.profile_reps):
        M.spmv(xd, yd)
    for _ in range(args.profile_reps):
        Cm.csr_spmv(xd, yd)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "done", "workload": wl, "n": A.nrows, "nnz": A.nnz,
                      "bandwidth": e["w"], "copy_bytes": 1 << 30, "da": args.profile_da,
                      "csr": args.profile_csr, "cache": args.profile_cache}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tune-reps", type=int, default=10)
    ap.add_argument("--dump", default=None, help="write the autotuner's timing table here (JSON)")
    ap.add_argument("--skip-banded", action="store_true", help="skip the random banded workload")
    ap.add_argument("--skip-cg", action="store_true", help="skip the conjugate-gradient solves")
    ap.add_argument("--skip-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--skip-sweep", action="store_true", help="skip the 27-point size sweep")
    ap.add_argument("--skip-cube", action="store_true", help="skip the 256^3 CSR CG solves")
    ap.add_argument("--skip-grid", action="store_true",
                    help="skip the index / scalar width grid and the non-square products")
    ap.add_argument("--skip-blocks", action="store_true", help="skip the DA-BSR / BSR products")
    ap.add_argument("--skip-coo", action="store_true", help="skip the DA-COO / COO products")
    ap.add_argument("--skip-spmm", action="store_true", help="skip the SpMM products")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-workgroups", type=int, default=0)
    ap.add_argument("--profile", action="store_true",
                    help="short run for counter collection: copy probe, then DA and CSR SpMV "
                         "with the launch shapes of --profile-da and --profile-csr")
    ap.add_argument("--da-launch", default=None,
                    help="DA-CSR launch shape of the main product (stream_gG_tT or paired_gG_tT); "
                         "default: autotuned")
    ap.add_argument("--csr-launch", default=None,
                    help="CSR launch shape of the comparison (stream_gG_tT or paired_gG_tT); "
                         "default: autotuned")
    ap.add_argument("--profile-da", default="stream_g2_t1024",
                    help="DA-CSR launch shape of the counter run")
    ap.add_argument("--profile-csr", default="stream_g2_t1024",
                    help="CSR launch shape of the counter run")
    ap.add_argument("--profile-workload", default="27pt",
                    help="matrix of the counter run: 27pt (128^3), band (n 4M, natural order), "
                         "band_rcm (the scrambled band after RCM + refinement), sweepN (the "
                         "27-point N^3 matrix), or readMB (only the read probe on an MB-sized "
                         "buffer, every read path, 20 launches of one pass and 5 of "
                         "1024 // MB passes each)")
    ap.add_argument("--profile-cache", default="nt", choices=("nt", "plain"),
                    help="cache policy of the matrix stream in the counter run")
    ap.add_argument("--profile-reps", type=int, default=10,
                    help="launches of each product in the counter run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2307_06305_amd as D
    from paper_2307_06305_amd.tuning import autotune, candidates, config_name
    from workloads import config_description, config_matrix, config_vector

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name}, {props.multi_processor_count} CUs")

    if args.profile:
        profile_run(D, args)
        return

    t = time.time()
    A = config_matrix(1)
    log(f"matrix {A.name}: n={A.nrows} nnz={A.nnz} ({time.time() - t:.1f}s)")
    t = time.time()
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=True)
    log(f"encode: w={e['w']} permuted={e['permuted']} ({time.time() - t:.1f}s)")
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    x = config_vector(1, A.ncols)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.zeros(A.nrows, dtype=torch.float64, device=dev)
    yc = torch.zeros_like(yd)

    # streaming ceiling: 2 GiB read along the products' own path (direct-to-LDS
    # 16-byte loads, non-temporal, 8 KiB tiles)
    buf = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    sink = torch.zeros(65536, dtype=torch.float64, device=dev)
    t_read = epochs(lambda: D.stream_read(buf, sink, D.READ_LDS_NT, 8192), 10, 3)
    stream_gbs = buf.numel() / t_read / 1e9
    del buf
    log(f"streaming read ceiling: {stream_gbs:.0f} GB/s")
    # the product's x gathers alone: the 27 DA offsets of the stencil for
    # every row, no matrix stream
    N = 128
    offs27 = torch.tensor([dz * N * N + dy * N + dx for dz in (-1, 0, 1) for dy in (-1, 0, 1)
                           for dx in (-1, 0, 1)], dtype=torch.int32, device=dev)

    # pick launch shapes (autotuner), unless given: a kernel trace of a run
    # with fixed shapes holds only the timed launches of each product
    from paper_2307_06305_amd.profiling import stream_launch

    def pick(mat, y, given):
        if given is None:
            return autotune(mat, xd, y, reps=args.tune_reps)
        g, t, u = stream_launch(given)
        cfg = (D.VAR_STREAM, g, u, t)
        mat.set_config(*cfg)
        time_launches(lambda: mat.apply(xd, y), 200)  # a sustained run, as the tuner ends with
        return cfg, {cfg: float("nan")}

    # CSR first: the tuner ends with a sustained run of its choice, so the
    # timed DA-CSR steps below follow a sustained run of their own kernel
    best_csr, times_csr = pick(Cm, yc, args.csr_launch)
    best_da, times_da = pick(M, yd, args.da_launch)
    log(f"DA best {config_name(best_da)} {times_da[best_da]*1e6:.1f}us; "
        f"CSR best {config_name(best_csr)} {times_csr[best_csr]*1e6:.1f}us")
    if args.dump:
        with open(args.dump, "w") as f:
            json.dump({"da": {config_name(c): t * 1e6 for c, t in sorted(times_da.items(), key=lambda kv: kv[1])},
                       "csr": {config_name(c): t * 1e6 for c, t in sorted(times_csr.items(), key=lambda kv: kv[1])}},
                      f, indent=1)

    T_da = model_bytes(A.nrows, A.ncols, A.nnz, 2)
    T_csr = model_bytes(A.nrows, A.ncols, A.nnz, 4)

    # timed region: K DA-CSR SpMVs
    for _ in range(args.warmup):
        M.spmv(xd, yd)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        M.spmv(xd, yd)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    t_da_events = start.elapsed_time(stop) * 1e-3 / args.steps
    ms_per_step = wall * 1e3 / args.steps

    # comparison path and repeat measurement (min over epochs)
    t_da = epochs(lambda: M.spmv(xd, yd), 50)
    t_csr = epochs(lambda: Cm.csr_spmv(xd, yc), 50)
    t_gather = epochs(lambda: D.gather_read(xd, sink, A.nrows, 27, offs=offs27), 50)

    # correctness of the timed output against CSR on the same x
    torch.cuda.synchronize()
    diff = (yd - yc).abs().max().item()

    W = 2 * A.nnz + 2 * A.nrows
    da_gbs = T_da / t_da_events / 1e9
    # HBM bytes per launch from the recorded counter runs, while the kernel
    # sources are unchanged and the timed launch shape is the profiled one
    from paper_2307_06305_amd.profiling import read_traffic

    tb = None
    for name in ("spmv_27pt128_traffic.md", "spmv_27pt128_paired_traffic.md"):
        tb = read_traffic(os.path.join(ROOT, "profiles", name), "da", launch=config_name(best_da))
        if tb is not None:
            break
    traffic = None if tb is None else int(round(tb))
    res = {
        "metric": "DA-CSR vs CSR SpMV effective GB/s, % HBM peak, speedup; CG time to 1e-10",
        "value": round(T_da / (ms_per_step * 1e-3) / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": config_description(1), "n": A.nrows, "nnz": A.nnz,
                   "bandwidth": e["w"], "index": "int16 DA offsets", "values": "f64",
                   "launch": config_name(best_da)},
        "roofline": {"bound": "hbm", "achieved": round(da_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(da_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "da": {"us": round(t_da * 1e6, 2), "model_bytes": T_da,
               "gbs": round(T_da / t_da / 1e9, 1),
               "pct_hbm_peak": round(100 * T_da / t_da / 1e9 / HBM_PEAK_GBS, 2),
               "gflops": round(W / t_da / 1e9, 1), "launch": config_name(best_da)},
        "csr": {"us": round(t_csr * 1e6, 2), "model_bytes": T_csr,
                "gbs": round(T_csr / t_csr / 1e9, 1),
                "pct_hbm_peak": round(100 * T_csr / t_csr / 1e9 / HBM_PEAK_GBS, 2),
                "gflops": round(W / t_csr / 1e9, 1), "launch": config_name(best_csr)},
        "speedup": round(t_csr / t_da, 4),
        "predicted_speedup": round(T_csr / T_da, 4),
        "uplift_fraction": round((t_csr / t_da - 1) / (T_csr / T_da - 1), 3),
        "stream_read_gbs": round(stream_gbs, 1),
        # additive bound: the matrix stream at the read ceiling plus the x
        # gathers alone (the two share each CU's vector memory path)
        "gather_probe_us": round(t_gather * 1e6, 2),
        "bound_us": round((T_da / (stream_gbs * 1e9) + t_gather) * 1e6, 2),
        "max_abs_diff_da_vs_csr": diff,
        "paper_cpu_context": {"uplift_st": 0.11, "uplift_mt": 0.175, "predicted": 0.20},
    }

    if not args.skip_banded:
        res["banded"] = bench_banded(D, args)
    if not args.skip_cg:
        res["cg"] = bench_cg(D, args)
    if not args.skip_cube:
        res["cg_cube"] = bench_cg_cube(D, args)
    if not args.skip_sweep:
        res["mall"] = bench_mall(D, args)
        res["sweep"] = bench_sweep(D, args)
    if not args.skip_grid:
        res["grid"] = bench_grid(D, args)
    if not args.skip_blocks:
        res["blocks"] = bench_blocks(D, args)
    if not args.skip_spmm:
        res["spmm"] = bench_spmm(D, args)
    if not args.skip_coo:
        res["coo"] = bench_coo(D, args)
    if not args.skip_batch:
        res["batch"] = bench_batch(D, args)
        res["selector_training"] = bench_selector_training(D, args)

    if not args.no_cpu:
        res["cpu_native"] = cpu_native(A, e, x)
        t_cpu, reps = cpu_baseline(A, e, x)
        res["cpu_baseline"] = {
            "value": round(T_da / t_cpu / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle DA-CSR SpMV (NumPy, float64) on the full workload, {reps} runs, "
                      f"{t_cpu:.2f} s each",
        }
    print(json.dumps(res), flush=True)
    summary(res)


if __name__ == "__main__":
    main()
