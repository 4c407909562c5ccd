"""Throughput of the batched Whittaker-Henderson smoother on one MI355X.

One step = one forward solve (``whs_solve``) plus one adjoint
(``whs_backward``) over the whole batch, inputs resident in HBM.  The
default workload is the heteroscedastic one: P = 65,536 series, T = 3288
daily steps (2016-2024), order d = 2, one band, one smoothing weight per
difference row (a GP field in log10), FP32 storage with FP64 arithmetic.

Prints one JSON line.  ``roofline`` covers the dominant kernel (the
adjoint), timed with HIP events on the stream it runs on; ``cpu_baseline``
times the FP64 CPU oracle on a bounded sample of the same inputs.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "series/sec (T=3288,d=2,fwd+bwd) and % of HBM roofline; held-out RMSE vs plain"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64
# FP64 operations (an FMA counts two) of one step of the GCV kernel's forward
# recurrence and its derivative along W, per grid value, at d = 1..4
GCV_FLOPS_PER_STEP = {1: 31, 2: 50, 3: 75, 4: 106}


def alg_bytes(T: int, d: int, C: int, esz: int, per_diff: bool, w_bits: bool = False):
    """Algorithmic HBM bytes per series: every API tensor once per pass at its dtype
    (the 0/1 weights one byte per day, or one bit when packed)."""
    lam = esz * (T - d) if per_diff else esz
    wb = T / 8 if w_bits else T
    fwd = esz * T * C + wb + lam + esz * T * C                        # x, w, lambda in; z out
    bwd = esz * T * C + wb + lam + esz * T * C + esz * T * C + lam    # g, w, lambda, z in; grad_x, grad_lambda out
    return fwd, bwd


# Sources of the two-sweep kernels whose HBM counters profiles/traffic.json holds.
TRAFFIC_SOURCES = ("whs_step.h", "whs_fast.h", "whs_two_sweep.h", "whs_kernels.h", "whs_dispatch.hip",
                   "inst_solve_d2.hip", "inst_backward_d2.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2604_00048_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    if none exists for this kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    e = rec.get(f"{kernel}|{workload}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def _counter_rows(root: str):
    """(kernel name, counter name, value) of every dispatch in rocprofv3's csv output under ``root``."""
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                out.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return out


def _mean_counter(rows, name_part: str, counter: str):
    vals = [v for k, c, v in rows if name_part in k and c == counter]
    if not vals:
        raise SystemExit(f"no {counter} samples for kernels matching {name_part!r}")
    return sum(vals) / len(vals), len(vals)


def ingest_counters(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, P, T, d, w_bits=False):
    """HBM bytes per launch of the two headline kernels from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the counter reads for a plain 256 MiB
    device copy (``--calibrate-copy``)."""
    copy_kib = (256 << 20) / 1024
    cf, _ = _mean_counter(_counter_rows(cal_fetch_dir), "copy", "FETCH_SIZE")
    cw, _ = _mean_counter(_counter_rows(cal_write_dir), "copy", "WRITE_SIZE")
    fs, ws = copy_kib / cf, copy_kib / cw
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    workload = f"heteroscedastic P={P} T={T} d={d} C=1" + (" w bits" if w_bits else "")
    fb, bb = alg_bytes(T, d, 1, 4, True, w_bits)
    rec = {}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
    print(f"calibration: copy of 256 MiB reads FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB "
          f"-> scales {fs:.3f} / {ws:.3f}")
    print("| API call | kernel | dispatches | algorithmic GB | HBM read GB | HBM write GB | traffic / algorithmic |")
    print("|---|---|---|---|---|---|---|")
    for call, bwd, alg in (("whs_solve", "false", fb), ("whs_backward", "true", bb)):
        # k_fast<d, 1 band, tile, float, adjoint?, per-difference weights, uneven dates?, weights as bits?>
        part = f"k_fast<{d}, 1, "
        tail = f"float, {bwd}, true, false, {'true' if w_bits else 'false'}>"
        names = sorted({k for k, c, v in fr if part in k and tail in k})
        if len(names) != 1:
            raise SystemExit(f"expected one {call} kernel, found {names}")
        kname = names[0]
        f_kib, n = _mean_counter(fr, kname, "FETCH_SIZE")
        w_kib, _ = _mean_counter(wr, kname, "WRITE_SIZE")
        rd, wt = f_kib * 1024 * fs, w_kib * 1024 * ws
        rec[f"{call}|{workload}"] = {"source_hash": kernel_source_hash(), "kernel": kname,
                                     "bytes_per_launch": rd + wt, "read_bytes": rd, "write_bytes": wt,
                                     "fetch_scale": fs, "write_scale": ws}
        print(f"| {call} | `{kname}` | {n} | {alg * P / 1e9:.3f} | {rd / 1e9:.3f} | {wt / 1e9:.3f} | "
              f"{(rd + wt) / (alg * P):.2f} |")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {path} (kernel source hash {kernel_source_hash()})")


def _cpu_worker(args):
    import numpy as np
    from oracle import whs_ref as R
    x, w, lam, g, d = args
    z, _ = R.solve_band(x, w, lam, d)
    R.vjp(x, w, lam, d, g, z=z)
    return x.shape[0]


def _lapack_worker(args):
    """Forward + adjoint of a chunk of series with LAPACK's banded SPD solver (dpbsv)."""
    import numpy as np
    import scipy.linalg
    from oracle import whs_ref as R
    x, w, lam, g, d = args
    AB = R.omega_band(w, lam, d)
    for p in range(x.shape[0]):
        z = scipy.linalg.solveh_banded(AB[p], np.where(w[p] != 0, x[p], 0.0), lower=True)
        u = scipy.linalg.solveh_banded(AB[p], g[p], lower=True)
        _ = np.where(w[p] != 0, u, 0.0)
        _ = -(R.apply_D(u[None], d) * R.apply_D(z[None], d))
    return x.shape[0]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pk, d: int, n_sample: int, workers: int, worker=None):
    """Time the FP64 oracle (forward + adjoint) on ``n_sample`` series of the same
    inputs, split over ``workers`` processes."""
    import multiprocessing as mp

    import numpy as np
    import torch

    idx = torch.arange(n_sample)
    b = pk.series(idx)
    x = b.x.numpy()[:, :, 0]
    w = b.w.numpy()
    lam = b.lam.numpy()
    g = np.random.default_rng(0).normal(size=x.shape)
    chunks = np.array_split(np.arange(n_sample), workers)
    jobs = [(x[c], w[c], lam[c], g[c], d) for c in chunks if len(c)]
    fn = worker or _cpu_worker
    ctx = mp.get_context("fork")
    with ctx.Pool(len(jobs)) as pool:
        pool.map(fn, [(j[0][:2], j[1][:2], j[2][:2], j[3][:2], d) for j in jobs])  # warm imports
        t0 = time.perf_counter()
        done = sum(pool.map(fn, jobs))
        dt = time.perf_counter() - t0
    return done / dt, dt, len(jobs)


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def bench_multiband(args):
    """Homoscedastic, ten bands sharing one factor, forward solve."""
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    P, T, C, d, S = args.P, args.T, 10, 2, args.interleave
    pk = synth.generate_packed("multiband", P, S=S, dtype=dtype, device=dev, chunk=8192, T=T, C=C)
    z = torch.empty_like(pk.x)
    info = torch.empty(P, dtype=torch.int32, device=dev)
    desc = whs.make_desc(P, T, d, C, S, whs.WHS_F64 if dtype == torch.float64 else whs.WHS_F32, whs.WHS_LAMBDA_SCALAR)
    ws = torch.empty(whs.workspace_bytes(desc), dtype=torch.uint8, device=dev)
    if args.fwd_bwd:
        # the adjoint too, against a seeded upstream gradient: g, grad_x, grad_lambda
        g = torch.randn(pk.x.shape, generator=torch.Generator(device=dev).manual_seed(7), device=dev, dtype=dtype)
        gx = torch.empty_like(pk.x)
        gl = torch.empty(P, dtype=dtype, device=dev)

    def step():
        whs.whs_solve(pk.x, pk.w, pk.lam, d, P, z=z, info=info, workspace=ws)
        if args.fwd_bwd:
            whs.whs_backward(pk.w, pk.lam, z, g, d, P, grad_x=gx, grad_lambda=gl, info=info, workspace=ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = _events(2)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    esz = 8 if dtype == torch.float64 else 4
    fb, bb = alg_bytes(T, d, C, esz, False)
    if args.fwd_bwd:
        fb += bb
    gbs = fb * P / (ms * 1e-3) / 1e9
    return {
        "metric": f"series/sec (T=3288,d=2,C=10 {'fwd+bwd' if args.fwd_bwd else 'forward'})", "value": P / (ms * 1e-3),
        "unit": "series/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"homoscedastic smoother {'fwd+bwd' if args.fwd_bwd else 'forward'}: P={P}, T={T}, "
                               f"d=2, C=10 bands sharing one factor, "
                               f"scalar lambda, {'FP64' if args.dtype == 'f64' else 'FP32'} storage / "
                               f"FP64 arithmetic",
                   "P": P, "T": T, "d": d, "C": C, "storage": args.dtype},
        "roofline": {"bound": "hbm", "kernel": "whs_solve + whs_backward" if args.fwd_bwd else "whs_solve",
                     "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None, "alg_bytes_per_series": fb, "ms_per_launch": ms},
        "failed_series": int((info != 0).sum().item()),
    }


def bench_uneven(args):
    """Uneven lengths and orders in one persistent launch, replayed from a HIP graph."""
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    groups = synth.uneven_groups(n_series=args.n_uneven, device=dev)
    x, w, lam, descs = synth.pack_groups(groups, dtype=torch.float32, device=dev)
    z = torch.empty_like(x)
    N = sum(d_["n_series"] for d_ in descs)
    info = torch.empty(N, dtype=torch.int32, device=dev)
    plan = whs.Plan(descs, torch.float32)
    cfg = plan.autotune(w, lam, x, z, force=args.retune)
    for _ in range(args.warmup):
        plan.graph_launch(w, lam, x, z, info)
    torch.cuda.synchronize()
    e0, e1 = _events(2)
    e0.record()
    for _ in range(args.steps):
        plan.graph_launch(w, lam, x, z, info)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    alg = sum(d_["n_series"] * (4 * d_["T"] + d_["T"] + 4 + 4 * d_["T"]) for d_ in descs)
    gbs = alg / (ms * 1e-3) / 1e9
    longest = max(d_["T"] for d_ in descs)
    return {
        "metric": "series/sec (uneven T in {365,730,1461,3288}, d in {1,2,3}, forward, one persistent launch)",
        "value": N / (ms * 1e-3), "unit": "series/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"uneven batch: {N} series, T in {{365,730,1461,3288}}, d in {{1,2,3}}, scalar "
                               f"lambda, FP32 storage, HIP-graph replay of one persistent launch",
                   "n_series": N, "groups": len(descs), "plan": cfg, "longest_T": longest},
        "roofline": {"bound": "hbm", "kernel": "whs_plan", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None, "alg_bytes": alg, "ms_per_launch": ms},
        "failed_series": int((info != 0).sum().item()),
    }


def bench_gcv(args):
    """The plain form: a scalar weight per series by GCV over 21 grid values
    (10^-1 .. 10^5), then the solve at the chosen weight."""
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    P, T, d, S = args.P, args.T, args.d, args.interleave
    pk = synth.generate_packed("multiband", P, S=S, dtype=dtype, device=dev, chunk=8192, T=T, C=1)
    grid = torch.tensor([10.0 ** (-1.0 + 0.3 * i) for i in range(21)], dtype=torch.float64, device=dev)
    lam_best = torch.empty(P, dtype=dtype, device=dev)
    info = torch.empty(P, dtype=torch.int32, device=dev)
    z = torch.empty_like(pk.x)
    desc = whs.make_desc(P, T, d, 1, S, whs.WHS_F64 if dtype == torch.float64 else whs.WHS_F32, whs.WHS_LAMBDA_SCALAR)
    nws = whs.workspace_bytes(desc)
    if S == 1:
        # series-contiguous: one workspace for the copies of both calls
        nws = max(nws, int(whs.lib().whs_interleave_workspace_bytes(ctypes.byref(desc))))
    ws = torch.empty(max(nws, 8), dtype=torch.uint8, device=dev)
    ev = _events(2 * args.steps + 2)

    def step(k=None):
        if k is not None:
            ev[2 * k].record()
        whs.whs_gcv(pk.x, pk.w, grid, d, P, lambda_best=lam_best, info=info, workspace=ws)
        if k is not None:
            ev[2 * k + 1].record()
        whs.whs_solve(pk.x, pk.w, lam_best, d, P, z=z, workspace=ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = ev[-2], ev[-1]
    e0.record()
    for k in range(args.steps):
        step(k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gcv_ms = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)) / args.steps
    flops = GCV_FLOPS_PER_STEP[d] * T * grid.numel() * P
    tf = flops / (gcv_ms * 1e-3) / 1e12
    return {
        "metric": f"series/sec (GCV over 21 weights + solve, T={T}, d={d})", "value": P / (ms * 1e-3),
        "unit": "series/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plain form: GCV choice of a scalar weight over 21 grid values, then the solve at "
                               f"it: P={P} series, T={T} daily steps, d={d}, one band, "
                               f"{'FP64' if args.dtype == 'f64' else 'FP32'} storage / FP64 arithmetic",
                   "P": P, "T": T, "d": d, "n_grid": grid.numel(), "storage": args.dtype, "interleave": S,
                   **({"contiguous_path": "interleaved copies"} if S == 1 else {})},
        "roofline": {"bound": "alu", "kernel": "whs_gcv", "achieved": tf, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS, "traffic": None,
                     "flops_per_series_step_grid_value": GCV_FLOPS_PER_STEP[d], "ms_per_launch": gcv_ms},
        "mean_log10_lambda": float(torch.log10(lam_best.double()).mean().item()),
        "failed_series": int((info != 0).sum().item()),
    }


def bench_variance(args):
    """Posterior variance diag(Omega^-1) of the heteroscedastic batch (0/1 weights,
    a weight per difference row): the two sweeps without a right-hand side."""
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    f64 = args.dtype == "f64"
    dt, esz = (torch.float64, 8) if f64 else (torch.float32, 4)
    d, S, P, T = args.d, args.interleave, args.P, args.T
    pk = synth.generate_packed("heteroscedastic", P, S=S, dtype=dt, device=dev, chunk=8192, T=T, d=d)
    desc = whs.make_desc(P, T, d, 1, S, whs.WHS_F64 if f64 else whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    nws = int(whs.lib().whs_variance_workspace_bytes(ctypes.byref(desc)))
    ws = torch.empty(max(nws, 8), dtype=torch.uint8, device=dev)
    var = torch.empty_like(pk.x)
    info = torch.empty(P, dtype=torch.int32, device=dev)

    def step():
        whs.whs_variance(pk.w, pk.lam, d, P, var=var, info=info, workspace=ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = _events(2)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    alg = T + esz * (T - d) + esz * T      # w, lambda, var: each once
    gbs = alg * P / (ms * 1e-3) / 1e9
    return {
        "metric": f"series/sec (posterior variance, T={T}, d={d})", "value": P / (ms * 1e-3),
        "unit": "series/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"posterior variance diag(Omega^-1): P={P} series, T={T} daily steps, d={d}, "
                               f"per-difference lambda (log10 GP field), {'FP64' if f64 else 'FP32'} storage / "
                               f"FP64 arithmetic", "P": P, "T": T, "d": d, "storage": args.dtype, "interleave": S,
                   **({"contiguous_path": "interleaved copies"} if S == 1 else {})},
        "roofline": {"bound": "hbm", "kernel": "whs_variance", "achieved": gbs, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None, "alg_bytes_per_series": alg,
                     "ms_per_launch": ms},
        "failed_series": int((info != 0).sum().item()),
    }


def bench_uneven_dates(args):
    """Forward solve + adjoint on irregular acquisition dates (the divided-difference
    D of the real dates, through its coefficient table): P series sharing --acq dates,
    --bands bands each, a weight per difference row, FP32 storage."""
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    P, T, C, d = args.P, args.acq, args.bands, args.d
    S, n = 64, 8192
    if P % n:
        raise SystemExit(f"--P must be a multiple of {n} for this workload")
    gen = torch.Generator(device=dev).manual_seed(23)
    days = synth.acquisition_days(T, gen, dev)
    coef = whs.whs_diff_coef(days.contiguous(), d)
    nb = P // S
    x = torch.empty((nb, T, C, S), dtype=torch.float32, device=dev)
    w = torch.empty((nb, T, S), dtype=torch.uint8, device=dev)
    for k in range(P // n):
        _, b = synth.irregular_sits(n, T, C, 29, dev, chunk=k, days=days)
        x[k * n // S:(k + 1) * n // S] = synth.pack_series(b.x.float(), S)
        w[k * n // S:(k + 1) * n // S] = synth.pack_rows(b.w, S)
        del b
    # log10 of the weight per difference row: uniform on [1, 4]
    lam = torch.pow(10.0, 1.0 + 3.0 * torch.rand((nb, T - d, S), generator=gen, device=dev)).float()
    g = torch.randn(x.shape, generator=gen, device=dev, dtype=torch.float32)
    z, gx, gl = torch.empty_like(x), torch.empty_like(x), torch.empty_like(lam)
    info = torch.empty(P, dtype=torch.int32, device=dev)
    desc = whs.make_desc(P, T, d, C, S, whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    ws = torch.empty(max(whs.workspace_bytes(desc), 8), dtype=torch.uint8, device=dev)

    def solve():
        whs.whs_solve(x, w, lam, d, P, z=z, info=info, workspace=ws, coef=coef)

    def adjoint():
        whs.whs_backward(w, lam, z, g, d, P, grad_x=gx, grad_lambda=gl, info=info, workspace=ws, coef=coef)
    for _ in range(args.warmup):
        solve()
        adjoint()
    torch.cuda.synchronize()
    K = args.steps
    ev = [_events(3) for _ in range(K)]
    e0, e1 = _events(2)
    e0.record()
    for k in range(K):
        ev[k][0].record()
        solve()
        ev[k][1].record()
        adjoint()
        ev[k][2].record()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / K
    bwd_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / K
    fb, bb = alg_bytes(T, d, C, 4, True)
    fwd_gbs, bwd_gbs = fb * P / (fwd_ms * 1e-3) / 1e9, bb * P / (bwd_ms * 1e-3) / 1e9
    step_gbs = (fb + bb) * P / (ms * 1e-3) / 1e9
    return {
        "metric": f"series/sec (uneven dates, T={T} acquisitions, C={C} bands, d={d}, fwd+bwd)",
        "value": P / (ms * 1e-3), "unit": "series/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"smoother fwd+bwd on irregular acquisition dates: P={P} series sharing T={T} "
                               f"dates over 3288 days, C={C} bands (double-logistic phenology, Bernoulli validity "
                               f"masks), d={d}, per-difference lambda, FP32 storage / FP64 arithmetic",
                   "P": P, "T": T, "C": C, "d": d, "storage": "f32", "interleave": S},
        "roofline": {"bound": "hbm", "kernel": "whs_backward_coef", "achieved": bwd_gbs, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": bwd_gbs / PEAK_HBM_GBS, "traffic": None, "alg_bytes_per_series": bb,
                     "ms_per_launch": bwd_ms},
        "kernels": {
            "whs_solve_coef": {"ms": fwd_ms, "alg_GBps": fwd_gbs, "frac": fwd_gbs / PEAK_HBM_GBS,
                               "alg_bytes_per_series": fb},
            "whs_backward_coef": {"ms": bwd_ms, "alg_GBps": bwd_gbs, "frac": bwd_gbs / PEAK_HBM_GBS},
            "step": {"ms": ms, "alg_GBps": step_gbs, "frac": step_gbs / PEAK_HBM_GBS},
        },
        "failed_series": int((info != 0).sum().item()),
    }


def bench_learned(args):
    """Learned per-day weights vs the GCV-chosen scalar weight, held-out RMSE and throughput."""
    import torch
    from paper_2604_00048_amd import learned
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    L = learned.train(dev, steps=args.train_steps, batch_size=4096, lr=args.lr, clouds=args.clouds,
                      log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    Ls = learned.train_scalar(dev, steps=args.train_steps, batch_size=4096, clouds=args.clouds,
                              log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    ev = learned.evaluate(L, dev, n_series=args.eval_series, Ls=Ls, clouds=args.clouds)
    return {
        "metric": "held-out RMSE (learned per-day lambda vs GCV scalar lambda), T=3288, d=2",
        "value": ev["rmse_learned"], "unit": "reflectance RMSE", "n_gpus": 1, "steps": args.train_steps,
        "warmup": 0, "ms_per_step": t_train / max(args.train_steps, 1) * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": f"learned weights (per-day network, and one shared weight for the homoscedastic "
                               f"model): 4-layer conv net (kernel 9, 64 channels, BF16 MFMA) trained "
                               f"{args.train_steps} steps of 4096 series through the smoother, evaluated on "
                               f"{args.eval_series} fresh series against GCV over 21 scalar weights",
                   "train_steps": args.train_steps, "lr": args.lr, "clouds": args.clouds},
        "heldout": ev,
        "train_seconds": t_train,
    }


def bench_transformer(args):
    """Heteroscedastic transformer weights vs one learned weight on irregular
    multi-band series through the uneven-date smoother: held-out RMSE and time."""
    import torch
    from paper_2604_00048_amd import learned_tf
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    het, hom, s_step = learned_tf.train(dev, steps=args.train_steps, batch_size=4096, lr=args.lr, T=args.acq,
                                        C=args.bands, clouds=args.clouds,
                                        log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = learned_tf.evaluate(het, hom, dev, n_series=args.eval_series, T=args.acq, C=args.bands, clouds=args.clouds)
    return {
        "metric": f"held-out RMSE (transformer per-acquisition lambda vs one learned lambda), T={args.acq} uneven "
                  f"dates, C={args.bands}, d=2",
        "value": ev["rmse_hetero_transformer"], "unit": "reflectance RMSE", "n_gpus": 1, "steps": args.train_steps,
        "warmup": 0, "ms_per_step": s_step * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": f"heteroscedastic vs homoscedastic smoothing of irregular series: 2-layer "
                               f"transformer (width 64, 2 heads, sinusoidal date encoding, BF16 MFMA products) "
                               f"trained {args.train_steps} steps of 4096 series sharing {args.acq} acquisition "
                               f"dates, {args.bands} bands, through the uneven-date smoother; evaluated on "
                               f"{args.eval_series} fresh series",
                   "train_steps": args.train_steps, "lr": args.lr, "clouds": args.clouds},
        "heldout": ev,
        "train_seconds": t_train,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hetero",
                    choices=["hetero", "multiband", "uneven", "learned", "transformer", "gcv", "variance",
                             "uneven_dates"])
    ap.add_argument("--P", type=int, default=None)
    ap.add_argument("--T", type=int, default=3288)
    ap.add_argument("--d", type=int, default=2, help="difference order of the heteroscedastic workload")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--fwd-bwd", action="store_true", help="multiband workload: time the adjoint with the solve")
    ap.add_argument("--interleave", type=int, default=64)
    ap.add_argument("--w-bits", action="store_true", help="heteroscedastic workload: weights packed eight to a byte")
    ap.add_argument("--in-place", action="store_true",
                    help="interleave 1: read the contiguous layout in place instead of through interleaved copies")
    ap.add_argument("--n-uneven", type=int, default=100000)
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--clouds", type=float, default=0.0,
                    help="learned workload: fraction of acquisitions cloud-contaminated and kept as observed")
    ap.add_argument("--eval-series", type=int, default=None,
                    help="learned workloads: fresh series scored (262144, or 32768 for the transformer)")
    ap.add_argument("--acq", type=int, default=280, help="transformer workload: acquisitions per series")
    ap.add_argument("--bands", type=int, default=4, help="transformer workload: spectral bands")
    ap.add_argument("--heldout-steps", type=int, default=150,
                    help="default workload: training steps (4096 series each) of the learned form scored in 'heldout'")
    ap.add_argument("--heldout-series", type=int, default=65536,
                    help="default workload: fresh series on which the learned and GCV-plain forms are scored")
    ap.add_argument("--no-heldout", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="read rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv output of the default workload and of "
                         "--calibrate-copy, write profiles/traffic.json and print the per-kernel table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 256 MiB three times (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (pixels shard across GPUs "
                                   "with no exchange, see the design notes)"}), flush=True)
        sys.exit(2)

    if args.ingest_counters:
        P = args.P or 65536
        ingest_counters(*args.ingest_counters, P=P, T=args.T, d=args.d, w_bits=args.w_bits)
        return

    if args.calibrate_copy:
        import torch
        n = (256 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}))
        return

    import torch
    from paper_2604_00048_amd import whs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    whs.lib()
    if args.workload == "multiband":
        args.P = args.P or 262144
        print(json.dumps(bench_multiband(args)), flush=True)
        return
    if args.workload == "uneven":
        print(json.dumps(bench_uneven(args)), flush=True)
        return
    if args.workload == "gcv":
        args.P = args.P or 262144
        print(json.dumps(bench_gcv(args)), flush=True)
        return
    if args.workload == "uneven_dates":
        args.P = args.P or 262144
        print(json.dumps(bench_uneven_dates(args)), flush=True)
        return
    if args.workload == "variance":
        args.P = args.P or 65536
        print(json.dumps(bench_variance(args)), flush=True)
        return
    if args.workload == "learned":
        args.eval_series = args.eval_series or 262144
        print(json.dumps(bench_learned(args)), flush=True)
        return
    if args.workload == "transformer":
        args.eval_series = args.eval_series or 32768
        print(json.dumps(bench_transformer(args)), flush=True)
        return
    args.P = args.P or 65536
    print(json.dumps(bench_hetero(args)), flush=True)


def copy_ceiling(dev, nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Read+write GB/s of a plain device-to-device copy: the practical HBM ceiling on this GPU."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def bench_hetero(args):
    import torch
    from paper_2604_00048_amd import synth, whs
    dev = torch.device("cuda:0")
    d, S, P, T = args.d, args.interleave, args.P, args.T
    f64 = args.dtype == "f64"
    dt, esz = (torch.float64, 8) if f64 else (torch.float32, 4)
    t_gen = time.perf_counter()
    pk = synth.generate_packed("heteroscedastic", P, S=S, dtype=dt, device=dev, chunk=8192, T=T, d=d)
    g = torch.randn(pk.x.shape, generator=torch.Generator(device=dev).manual_seed(7), device=dev, dtype=dt)
    z = torch.empty_like(pk.x)
    gx = torch.empty_like(pk.x)
    gl = torch.empty_like(pk.lam)
    info = torch.empty(P, dtype=torch.int32, device=dev)
    desc = whs.make_desc(P, T, d, 1, S, whs.WHS_F64 if f64 else whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    nws = whs.workspace_bytes(desc)
    if S == 1 and not args.in_place:
        # series-contiguous: the workspace that runs the interleaved kernels on copies
        nws = max(nws, int(whs.lib().whs_interleave_workspace_bytes(ctypes.byref(desc))))
    ws = torch.empty(max(nws, 8), dtype=torch.uint8, device=dev)
    w_in = synth.pack_bits(pk.w) if args.w_bits else pk.w
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"# inputs generated in {t_gen:.1f}s; workspace {ws.numel() / 1e6:.1f} MB", file=sys.stderr, flush=True)

    def step():
        whs.whs_solve(pk.x, w_in, pk.lam, d, P, z=z, info=info, workspace=ws)
        whs.whs_backward(w_in, pk.lam, z, g, d, P, grad_x=gx, grad_lambda=gl, info=info, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for k in range(K):
        ev[k][0].record()
        whs.whs_solve(pk.x, w_in, pk.lam, d, P, z=z, info=info, workspace=ws)
        ev[k][1].record()
        whs.whs_backward(w_in, pk.lam, z, g, d, P, grad_x=gx, grad_lambda=gl, info=info, workspace=ws)
        ev[k][2].record()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / K
    bwd_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / K
    ms_step = total_ms / K
    step_ms = sorted(e[0].elapsed_time(e[2]) for e in ev)
    median_ms = step_ms[K // 2] if K % 2 else 0.5 * (step_ms[K // 2 - 1] + step_ms[K // 2])
    n_fail = int((info != 0).sum().item())

    print(f"# timed {K} steps: {total_ms / K:.3f} ms per step", file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling(dev)
    fb, bb = alg_bytes(T, d, 1, esz, True, args.w_bits)
    bwd_gbs = bb * P / (bwd_ms * 1e-3) / 1e9
    fwd_gbs = fb * P / (fwd_ms * 1e-3) / 1e9
    step_gbs = (fb + bb) * P / (ms_step * 1e-3) / 1e9
    workload = f"heteroscedastic P={P} T={T} d={d} C=1" + (" w bits" if args.w_bits else "") + (" f64" if f64 else "")
    traffic = measured_traffic("whs_backward", workload)
    out = {
        "metric": METRIC,
        "value": P / (ms_step * 1e-3),
        "unit": "series/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"heteroscedastic smoother fwd+bwd: P={P} series, T={T} daily steps, d={d}, C=1 band, "
                        f"per-difference lambda (log10 GP field), {'FP64' if f64 else 'FP32'} storage / FP64 arithmetic"
                        + (", 0/1 weights packed eight to a byte" if args.w_bits else ""),
            "P": P, "T": T, "d": d, "C": 1, "storage": args.dtype, "interleave": S,
            **({"w_format": "bits"} if args.w_bits else {}),
            **({"contiguous_path": "in place" if args.in_place else "interleaved copies"} if S == 1 else {}),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "whs_backward",
            "achieved": bwd_gbs,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": bwd_gbs / PEAK_HBM_GBS,
            "traffic": traffic,
            "alg_bytes_per_series": bb,
            "ms_per_launch": bwd_ms,
            "copy_GBps": copy_gbs,
        },
        "kernels": {
            "whs_solve": {"ms": fwd_ms, "alg_GBps": fwd_gbs, "frac": fwd_gbs / PEAK_HBM_GBS,
                          "alg_bytes_per_series": fb},
            "whs_backward": {"ms": bwd_ms, "alg_GBps": bwd_gbs, "frac": bwd_gbs / PEAK_HBM_GBS},
            "step": {"ms": ms_step, "median_ms": median_ms, "alg_GBps": step_gbs, "frac": step_gbs / PEAK_HBM_GBS},
        },
        "failed_series": n_fail,
        "wall_s_timed": wall,
        "build_id": whs.build_id(),
    }
    if not args.no_cpu_baseline:
        n = min(args.cpu_sample, P)
        workers = min(16, os.cpu_count() or 1, n)
        rate, secs, used = cpu_baseline(pk, d, n, workers)
        out["cpu_baseline"] = {
            "value": rate, "unit": "series/s", "cores": used, "kind": "oracle",
            "sample": f"{n} of the {P} series (first ones), FP64 numpy banded LDL^T forward + adjoint, "
                      f"{used} processes, {secs:.1f} s, host CPU {cpu_model()}",
        }
        nl = min(args.cpu_sample // 8, P)
        rate_l, secs_l, used_l = cpu_baseline(pk, d, nl, workers, worker=_lapack_worker)
        out["cpu_lapack"] = {
            "value": rate_l, "unit": "series/s", "cores": used_l, "kind": "LAPACK dpbsv (scipy solveh_banded)",
            "sample": f"{nl} of the {P} series, forward + adjoint solve per series, {used_l} processes, {secs_l:.1f} s",
        }
    if not args.no_heldout:
        out["heldout"] = heldout_clause(dev, args.heldout_steps, args.heldout_series)
    return out


def heldout_clause(dev, steps: int, n_series: int):
    """The metric's third clause, outside the timed region: the learned form (per-day
    weights from the convolution network) trained for a bounded number of steps
    through the smoother, then scored with the GCV-plain form on the same held-out
    points of fresh series, with each form's throughput (network + solve; GCV over
    21 weights + solve)."""
    import torch
    from paper_2604_00048_amd import learned
    t0 = time.perf_counter()
    L = learned.train(dev, steps=steps, batch_size=4096, lr=1e-3,
                      log=lambda m: print("# heldout " + m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = learned.evaluate(L, dev, n_series=n_series, chunk=min(n_series, 65536))
    ev.update({"train_steps": steps, "train_batch": 4096, "train_seconds": t_train,
               "note": "RMSE in data units over 10 % of the observed points of every fresh series, hidden from "
                       "both forms; series/s per form on chunks of up to 65,536 series"})
    return ev


if __name__ == "__main__":
    main()
