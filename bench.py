#!/usr/bin/env python3
"""Benchmark of the SGSPM time step on one MI355X.

Default workload: the 256x256x32 block (2.1 M cells, 4 nm cells, exchange +
anisotropy + stray field by zero-padded 512x512x64 FFT + rotating 10 mT field,
alpha = 1e-3, dt = 0.05 ps), FP32 bulk.  One "step" is one whole SGSPM step
(both Gauss-Seidel sweeps, damping, projection) over the grid; the metric is
cell-updates per second (cells x steps / wall) with inputs resident in HBM.

Also reported: the FP64 comparator on the same GPU, the adjoint step, the
per-kernel-class time and algorithmic bandwidth of the timed steps (HIP events
around every launch, a second timed pass), the dominant kernel against the HBM
roofline, the FP64 CPU oracle timed on the host, and the max |m - m_oracle| of
the first step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config block-256x256x32]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per SGSPM step (fwd, adjoint) FP32 vs FP64 at stated error; %HBM"
HBM_PEAK_GBS = 8000.0
# timing class -> kernel (rocprofv3 shows the float instance as sgspm::k_...<float>)
KERNEL_NAMES = {"row_fwd": "k_row_fwd", "row_fwd512": "k_row_fwd512", "row_inv": "k_row_inv",
                "row_inv512": "k_row_inv512", "col_dct": "k_col_dct",
                "yz_solve": "k_yz_solve", "yz_reg": "k_yz_reg", "col_fft": "k_col_fft", "fft512": "k_fft512",
                "conv": "k_conv", "conv64": "k_conv64", "other": "point-wise/reduction kernels"}
WORKLOAD_TEXT = {
    "block-256x256x32": "256x256x32 block, 4 nm cells, exchange+anisotropy+stray (padded 512x512x64 FFT)+rotating 10 mT, "
          "alpha 1e-3, dt 0.05 ps",
    "adjoint-film-128x128": "128x128x1 film, 4 nm cells, all fields, alpha 0.01, dt 0.1 ps",
    "wall-strip-512x32x4": "512x32x4 Neel-wall strip, 4 nm cells, all fields, 10 mT, alpha 1e-3, dt 0.1 ps",
    "film-128x64": "128x64x1 film, 4 nm cells, all fields, 5 mT, alpha 0.01, dt 0.1 ps",
    "mf-film-32x32": "32x32x1 exchange-only film, manufactured forcing off, alpha 0.01, dt 1e-3",
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_block-256x256x32.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2606_28113_amd", "csrc", f) for f in ("kernels.hip", "kernels.h", "fft_lds.h", "plan.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, dtype, workload):
    """HBM bytes per launch of `kernel` from the committed hardware-counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when the
    summary is absent, covers another workload, or the device sources (kernels, their
    launchers and the plan that sets their launch parameters) changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src = kernel_source_hash()
    for line in open(TRAFFIC_FILE):
        if not line.startswith("traffic:"):
            continue
        f = dict(kv.split("=", 1) for kv in line.split()[1:])
        if (f.get("kernel") == kernel and f.get("dtype") == dtype and f.get("workload") == workload
                and f.get("source_sha256") == src):
            return float(f["bytes_per_launch"])
    return None


def make_plan(sg, c, precision):
    kw = dict(nx=c.n[0], ny=c.n[1], nz=c.n[2], dx=c.h[0], dy=c.h[1], dz=c.h[2], dt=c.dt, precision=precision)
    if c.units == "si":
        kw.update(units=sg.UNITS_SI, A=c.A, Ms=c.Ms, Ku=c.Ku, terms=sg.TERM_ALL)
    else:
        kw.update(units=sg.UNITS_REDUCED, eps=c.eps, Q=c.Q, terms=sg.TERM_EXCHANGE)
    return sg.Plan(**kw)


def time_steps(torch, plan, m, alpha, B, first, count):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(first, first + count):
        plan.step(m, alpha, B[n])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / count


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="block-256x256x32")
    ap.add_argument("--fp64-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (hardware-counter calibration)")
    ap.add_argument("--copy-bw-mb", type=int, default=0,
                    help="first time 20 plain device copies of this many MiB (a practical HBM ceiling)")
    ap.add_argument("--skip-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures the single-GPU SGSPM step only; run it with --gpus 1 "
              "(sharding across GPUs is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2606_28113_amd as sg
    import workloads

    if args.copy_calib_mb:
        nb = args.copy_calib_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {nb} bytes read, {nb} bytes written", file=sys.stderr, flush=True)
        del src, dst
    if args.copy_bw_mb:
        nb = args.copy_bw_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        print(f"[bench] device copy of {args.copy_bw_mb} MiB: {us:.1f} us, {2 * nb / us / 1e3:.0f} GB/s read + write",
              file=sys.stderr, flush=True)
        del src, dst
    c = workloads.config(args.config)
    N = c.cells
    K, W = args.steps, args.warmup
    total = W + K + 1
    B = workloads.field_schedule(c, total)
    alpha = c.alpha
    m0 = workloads.initial_state(c)
    print(f"[bench] {c.name}: {c.n} cells={N} steps={K} warmup={W}", file=sys.stderr, flush=True)

    # ---- FP32 forward
    p32 = make_plan(sg, c, sg.FP32)
    m = torch.tensor(m0, dtype=torch.float32, device="cuda")
    p32.step(m, alpha, B[0])
    torch.cuda.synchronize()
    p32.check()
    m1_32 = m.detach().cpu().numpy().astype(np.float64)
    for n in range(1, 1 + W):
        p32.step(m, alpha, B[n])
    ms32 = time_steps(torch, p32, m, alpha, B, 1 + W, K)
    p32.check()
    print(f"[bench] fp32 forward {ms32:.4f} ms/step", file=sys.stderr, flush=True)
    # second timed pass with per-launch events
    p32.timing(True)
    for n in range(1 + W, 1 + W + K):
        p32.step(m, alpha, B[n])
    stats = p32.timing_read()
    p32.timing(False)
    breakdown = {}
    for k, (ms, by, cnt) in stats.items():
        if cnt:
            breakdown[KERNEL_NAMES[k]] = {"ms_per_step": ms / K, "launches_per_step": cnt / K,
                                          "avg_us": 1e3 * ms / cnt, "GBps": by / (ms * 1e-3) / 1e9,
                                          "alg_MB_per_launch": by / cnt / 1e6}
    dom = max(breakdown, key=lambda k: breakdown[k]["ms_per_step"])
    d = breakdown[dom]
    traffic = measured_traffic(dom, "f32", c.name)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(d["GBps"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_us": round(d["avg_us"], 3), "alg_bytes_per_launch": round(d["alg_MB_per_launch"] * 1e6)}
    alg_step_bytes = sum(stats[k][1] for k in stats) / K
    e32 = p32.energy(torch.tensor(m1_32, dtype=torch.float32, device="cuda"), B[0])
    del p32, m
    torch.cuda.empty_cache()

    # ---- FP64 forward (comparator on the same GPU)
    if args.skip_fp64:
        args.fp64_steps = 0
    p64 = make_plan(sg, c, sg.FP64)
    m = torch.tensor(m0, dtype=torch.float64, device="cuda")
    p64.step(m, alpha, B[0])
    torch.cuda.synchronize()
    m1_64 = m.detach().cpu().numpy()
    for n in range(1, 1 + min(W, 5)):
        p64.step(m, alpha, B[n])
    K64 = max(1, min(args.fp64_steps, K))
    ms64 = time_steps(torch, p64, m, alpha, B, 1 + min(W, 5), K64)
    p64.check()
    print(f"[bench] fp64 forward {ms64:.4f} ms/step", file=sys.stderr, flush=True)
    # per-kernel breakdown of the FP64 step (second pass with per-launch events)
    p64.timing(True)
    for n in range(1 + min(W, 5), 1 + min(W, 5) + K64):
        p64.step(m, alpha, B[n])
    stats64 = p64.timing_read()
    p64.timing(False)
    breakdown64 = {}
    for k, (ms, by, cnt) in stats64.items():
        if cnt:
            breakdown64[KERNEL_NAMES[k]] = {"ms_per_step": ms / K64, "launches_per_step": cnt / K64,
                                            "avg_us": 1e3 * ms / cnt, "GBps": by / (ms * 1e-3) / 1e9}

    # ---- adjoint step (FP32), if the library provides it
    adj = None
    try:
        if args.adjoint_steps <= 0:
            raise sg.SGSPMError(0, "adjoint timing skipped (--adjoint-steps 0)")
        pa = make_plan(sg, c, sg.FP32)
        ma = torch.tensor(m0, dtype=torch.float32, device="cuda")
        lam = torch.zeros_like(ma)
        grad = torch.zeros(4, dtype=torch.float64, device="cuda")
        pa.adjoint_step(ma, alpha, B[0], lam, grad)
        torch.cuda.synchronize()
        KA = args.adjoint_steps
        t0 = time.perf_counter()
        for n in range(KA):
            pa.adjoint_step(ma, alpha, B[n], lam, grad)
        torch.cuda.synchronize()
        msa = (time.perf_counter() - t0) * 1e3 / KA
        pa.timing(True)
        for n in range(KA):
            pa.adjoint_step(ma, alpha, B[n], lam, grad)
        stats_a = pa.timing_read()
        pa.timing(False)
        breakdown_a = {}
        for k, (ms, by, cnt) in stats_a.items():
            if cnt:
                breakdown_a[KERNEL_NAMES[k]] = {"ms_per_step": ms / KA, "launches_per_step": cnt / KA,
                                                "avg_us": 1e3 * ms / cnt, "GBps": by / (ms * 1e-3) / 1e9}
        adj = {"value": N / (msa * 1e-3), "unit": "cell-updates/s", "ms_per_step": msa, "steps": KA,
               "dtype": "f32", "note": "one adjoint step recomputes its forward step internally",
               "kernels": breakdown_a}
        del pa, ma, lam
    except sg.SGSPMError as e:
        adj = {"value": None, "note": str(e)}

    # ---- CPU oracle baseline and first-step error
    cpu = None
    err = {}
    if not args.no_cpu_baseline:
        from oracle import demag, scheme, units
        if c.units == "si":
            eps, Q, dtr, _ = units.reduce_si(c.A, c.Ms, c.Ku, c.dt)
            P = scheme.Problem(n=c.n, h=c.h, eps=eps, dt=dtr, Q=Q, stray=True)
            he = [units.field_from_tesla(b, c.Ms) for b in B[0]]
        else:
            P = scheme.Problem(n=c.n, h=c.h, eps=c.eps, dt=c.dt)
            he = list(B[0])
        P.spectra()
        S = 6 if N >= 1 << 20 else 20  # about 10-20 s of oracle work on 8 cores
        t0 = time.perf_counter()
        ref = np.asarray(m0, np.float64)
        first = None
        for n in range(S):
            ref = scheme.sgspm_step(P, ref, alpha, he if n == 0 else he)
            if first is None:
                first = ref
        tc = time.perf_counter() - t0
        cpu = {"value": S * N / tc, "unit": "cell-updates/s", "cores": demag.WORKERS, "kind": "oracle",
               "sample": f"{S} SGSPM steps of the same {c.n[0]}x{c.n[1]}x{c.n[2]} workload (FP64 NumPy/SciPy, "
                         f"FFT threads={demag.WORKERS}, tensor precompute excluded), {tc:.1f} s"}
        err["fp32_step1_max_abs"] = float(np.abs(m1_32 - first).max())
        err["fp64_step1_max_abs"] = float(np.abs(m1_64 - first).max())
        eref = scheme.energies(P, first, he)["total"] * (units.MU0 * c.Ms ** 2 if c.units == "si" else 1.0)
        err["fp32_step1_energy_rel"] = float(abs(e32["total"] - eref) / abs(eref))

    value = N / (ms32 * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c.name}: {WORKLOAD_TEXT[c.name]}", "cells": N, "global_batch": 1,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": {"value": N / (ms64 * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms64, "steps": K64,
                 "kernels": breakdown64},
        "adjoint": adj,
        "error_vs_oracle": err,
        "step_algorithmic_MB": alg_step_bytes / 1e6,
        "step_algorithmic_GBps": alg_step_bytes / (ms32 * 1e-3) / 1e9,
        "kernels": breakdown,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
