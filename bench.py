#!/usr/bin/env python3
"""Benchmark of the SGSPM time step on one MI355X.

Default workload: the 256x256x32 block (2.1 M cells, 4 nm cells, exchange +
anisotropy + stray field by zero-padded 512x512x64 FFT + rotating 10 mT field,
alpha = 1e-3, dt = 0.05 ps), FP32 bulk.  One "step" is one whole SGSPM step
(both Gauss-Seidel sweeps, damping, projection) over the grid; the metric is
cell-updates per second (cells x steps / wall) with inputs resident in HBM.

The forward step is timed over 5 passes of K steps each (HIP-stream
synchronisation around each pass); ms_per_step is the median pass.  Also
reported: the FP64 comparator on the same GPU, the adjoint step (FP32 and
FP64), the full checkpointed backward pass of the workload's adjoint length
(segment recompute included), the per-kernel-class time and launch-level
bandwidth of the timed steps (HIP events around every launch, a further timed
pass), the dominant kernel and the whole step against the HBM roofline on the
algorithmic byte count (each field read and written once per Gauss-Seidel
stage plus the demagnetising-tensor spectrum reads), the FP64 CPU oracle timed
on the host, and the max |m - m_oracle| of the first step.

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
    "wall-strip-512x32x4": "512x32x4 Neel-wall strip, 4 nm cells, all fields, 5 mT, alpha 0.01, dt 0.1 ps",
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


# Algorithmic bytes of one SGSPM step in single precision (double: twice): every
# field read once and written once per Gauss-Seidel stage A-F (stage A reads m2,
# m3 and writes g2, g3 and ... : 20 B per cell; B-E 28 each; F 32), 164 B per
# cell, plus the demagnetising-tensor spectrum: each output of a convolution
# reads its three tensor components once, 23 component reads per step (A: the
# outputs 2 and 3, five distinct components; B, C, D, E: one output, three; F:
# all six), each over the folded octant (nx+1)(ny+1)(nz+1).
FIELD_BYTES_PER_CELL = 164
TENSOR_READS_PER_STEP = 23
CONV_LAUNCHES_PER_STEP = 6


def algorithmic_step_bytes(c, dbytes):
    nx, ny, nz = c.n
    octant = (nx + 1) * (ny + 1) * (nz + 1 if nz > 1 else 1)
    field = FIELD_BYTES_PER_CELL * c.cells * dbytes // 4
    tensor = TENSOR_READS_PER_STEP * octant * dbytes
    return field, tensor


def make_plan(sg, c, precision, scheme=0, batch=0):
    kw = dict(nx=c.n[0], ny=c.n[1], nz=c.n[2], dx=c.h[0], dy=c.h[1], dz=c.h[2], dt=c.dt, precision=precision,
              scheme=scheme, batch=batch)
    if c.units == "si":
        kw.update(units=sg.UNITS_SI, A=c.A, Ms=c.Ms, Ku=c.Ku, terms=sg.TERM_ALL)
    else:
        kw.update(units=sg.UNITS_REDUCED, eps=c.eps, Q=c.Q, terms=sg.TERM_EXCHANGE)
    return sg.Plan(**kw)


def time_steps(torch, plan, m, alpha, B, first, count):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(first, first + count):
        plan.step(m, alpha, B[n % len(B)])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / count


def kernel_breakdown(stats, steps):
    out = {}
    for k, (ms, by, cnt) in stats.items():
        if cnt:
            out[KERNEL_NAMES[k]] = {"ms_per_step": ms / steps, "launches_per_step": cnt / steps,
                                    "avg_us": 1e3 * ms / cnt, "launch_level_GBps": by / (ms * 1e-3) / 1e9,
                                    "launch_level_MB_per_launch": by / cnt / 1e6}
    return out


def time_adjoint(torch, sg, c, precision, m0, B, alpha, KA):
    """ms per adjoint step (each recomputes its forward step) and its kernel breakdown."""
    pa = make_plan(sg, c, precision)
    dt_ = torch.float32 if precision == sg.FP32 else torch.float64
    ma = torch.tensor(m0, dtype=dt_, device="cuda")
    # a seeded random cotangent (the adjoint's arithmetic does not branch on values)
    lam = torch.tensor(np.random.default_rng(7).normal(size=m0.shape), dtype=dt_, device="cuda")
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    pa.adjoint_step(ma, alpha, B[0], lam, grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(KA):
        pa.adjoint_step(ma, alpha, B[n], lam, grad)
    torch.cuda.synchronize()
    msa = (time.perf_counter() - t0) * 1e3 / KA
    pa.timing(True)
    for n in range(KA):
        pa.adjoint_step(ma, alpha, B[n], lam, grad)
    stats = pa.timing_read()
    pa.timing(False)
    # the same adjoint step from a tape (the backward pass keeps its replayed steps' tapes)
    tape = pa.new_tapes(1)[0]
    mt = ma.clone()
    pa.step_taped(mt, alpha, B[0], tape)
    pa.adjoint_step_taped(ma, alpha, B[0], tape, lam, grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(KA):
        pa.adjoint_step_taped(ma, alpha, B[0], tape, lam, grad)
    torch.cuda.synchronize()
    mst = (time.perf_counter() - t0) * 1e3 / KA
    pa.close()
    return msa, kernel_breakdown(stats, KA), mst


def time_backward(torch, sg, c, precision, m0, alpha, S, K):
    """Forward with checkpoints every K steps and the full backward pass (segment
    replays with tapes plus S adjoint steps) of the terminal misfit L = mean (m_S - target)^2."""
    plan = make_plan(sg, c, precision)
    dt_ = torch.float32 if precision == sg.FP32 else torch.float64
    B = workloads.field_schedule(c, S)
    target = torch.tensor(workloads.target_state(c) if c.name in ("adjoint-film-128x128", "block-256x256x32")
                          else workloads.random_unit(c.shape, 51), dtype=dt_, device="cuda")
    m = torch.tensor(m0, dtype=dt_, device="cuda", requires_grad=True)
    he = torch.tensor(B, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    # an untimed pass of the same length first: the plan's adjoint workspace, the tapes,
    # the autograd engine and the allocator's blocks for every checkpoint and state start here
    sg.SGSPMFunction.apply(m, he, a, plan, K).sum().backward()
    m.grad = None
    he.grad = None
    a.grad = None
    torch.cuda.synchronize()
    # two timed passes (the first pass of a process runs 10-20% slower); the faster is reported
    fw, bw = [], []
    for _ in range(2):
        m.grad = None
        he.grad = None
        a.grad = None
        t0 = time.perf_counter()
        out = sg.SGSPMFunction.apply(m, he, a, plan, K)
        L = torch.mean((out - target) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fw.append((t1 - t0) * 1e3)
        bw.append((t2 - t1) * 1e3)
    plan.close()
    ok = bool(torch.isfinite(m.grad).all()) and bool(np.isfinite(float(a.grad)))
    return {"steps": S, "ckpt_every": K, "forward_ms": min(fw), "backward_ms": min(bw), "passes_backward_ms": bw,
            "backward_value": c.cells * S / (min(bw) * 1e-3), "unit": "cell-updates/s",
            "note": "backward = replay of every segment from its checkpoint, keeping each step's tape, "
                    "plus S adjoint steps from those tapes (each step runs forward once; the recompute "
                    "path when the tapes do not fit); value = cells x S / backward wall",
            "taped": bool(sg.autograd.TAPED),
            "grads_finite": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="block-256x256x32")
    ap.add_argument("--fp64-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--passes", type=int, default=5, help="timed passes of K steps (median reported)")
    ap.add_argument("--sweep-steps", type=int, default=5000,
                    help="steps per run of the strip workload's 15-run field/damping sweep (0: skip)")
    ap.add_argument("--metrics-log", default="",
                    help="write the sweep's per-run records (energies per term every 10 steps, max ||m| - 1|) "
                         "to this JSONL file")
    ap.add_argument("--backward-steps", type=int, default=-1,
                    help="steps of the timed checkpointed backward pass (-1: the workload's adjoint length, 0: skip)")
    ap.add_argument("--film-steps", type=int, default=200,
                    help="steps of the film-128x64 timing (0 skips the film workloads)")
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

    global np, workloads
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
    passes = []
    for _ in range(max(1, args.passes)):
        passes.append(time_steps(torch, p32, m, alpha, B, 1 + W, K))
    ms32 = float(np.median(passes))
    p32.check()
    print(f"[bench] fp32 forward {ms32:.4f} ms/step (median of {len(passes)} passes: "
          + ", ".join(f"{t:.4f}" for t in passes) + ")", file=sys.stderr, flush=True)
    # a further timed pass with per-launch events
    p32.timing(True)
    for n in range(1 + W, 1 + W + K):
        p32.step(m, alpha, B[n])
    stats = p32.timing_read()
    p32.timing(False)
    breakdown = kernel_breakdown(stats, K)
    dom = max(breakdown, key=lambda k: breakdown[k]["ms_per_step"])
    d = breakdown[dom]
    traffic = measured_traffic(dom, "f32", c.name)
    field_b, tensor_b = algorithmic_step_bytes(c, 4)
    launch_step_bytes = sum(stats[k][1] for k in stats) / K
    # the dominant kernel's share of the algorithmic bytes: the convolution reads
    # the tensor spectrum (its spectra are transform intermediates, not counted);
    # the other kernels move only intermediates or fields counted per stage
    if dom in ("k_conv64", "k_conv"):
        alg_launch = tensor_b / CONV_LAUNCHES_PER_STEP
    else:
        alg_launch = None
    avg_s = d["avg_us"] * 1e-6
    roofline = {"bound": "hbm", "kernel": dom,
                "achieved": round(alg_launch / avg_s / 1e9, 1) if alg_launch else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(alg_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4) if alg_launch else None,
                "traffic": traffic,
                "avg_launch_us": round(d["avg_us"], 3),
                "algorithmic_bytes_per_launch": round(alg_launch) if alg_launch else None,
                "launch_level_bytes_per_launch": round(d["launch_level_MB_per_launch"] * 1e6),
                "launch_level_GBps": round(d["launch_level_GBps"], 1),
                "launch_level_frac": round(d["launch_level_GBps"] / HBM_PEAK_GBS, 4),
                "step": {"algorithmic_bytes": field_b + tensor_b, "field_bytes": field_b, "tensor_bytes": tensor_b,
                         "GBps": round((field_b + tensor_b) / (ms32 * 1e-3) / 1e9, 1),
                         "frac": round((field_b + tensor_b) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "launch_level_bytes": round(launch_step_bytes),
                         "launch_level_GBps": round(launch_step_bytes / (ms32 * 1e-3) / 1e9, 1),
                         "launch_level_frac": round(launch_step_bytes / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
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
    breakdown64 = kernel_breakdown(stats64, K64)
    p64.close()
    del m
    torch.cuda.empty_cache()

    # ---- the frozen-field reading of the sweeps (two stray-field evaluations per step), FP32
    ff = None
    if c.units == "si":
        pf = make_plan(sg, c, sg.FP32, scheme=sg.SCHEME_SGS_FF)
        m = torch.tensor(m0, dtype=torch.float32, device="cuda")
        for n in range(1, 1 + min(W, 5)):
            pf.step(m, alpha, B[n])
        msf = float(np.median([time_steps(torch, pf, m, alpha, B, 1 + min(W, 5), K) for _ in range(3)]))
        pf.check()
        ff = {"value": N / (msf * 1e-3), "unit": "cell-updates/s", "ms_per_step": msf, "dtype": "f32",
              "note": "SGSPM with f frozen at m^n through both sweeps (stray field evaluated twice per step)"}
        print(f"[bench] fp32 frozen-field step {msf:.4f} ms/step", file=sys.stderr, flush=True)
        pf.close()
        del m
        torch.cuda.empty_cache()

    # ---- adjoint steps (FP32 and FP64) from a random cotangent at the workload's start
    adj = None
    if args.adjoint_steps > 0:
        KA = args.adjoint_steps
        adj = {"unit": "cell-updates/s", "steps": KA,
               "note": "one adjoint step recomputes its forward step internally; cotangent = seeded "
                       "N(0, 1) values, state = the workload's initial state; from_tape: the same step "
                       "from the tape of its forward step (sgspm_adjoint_step_taped, no recompute)"}
        for name, prec in (("f32", sg.FP32), ("f64", sg.FP64)):
            msa, bd, mst = time_adjoint(torch, sg, c, prec, m0, B, alpha, KA)
            adj[name] = {"value": N / (msa * 1e-3), "ms_per_step": msa, "kernels": bd,
                         "from_tape": {"value": N / (mst * 1e-3), "ms_per_step": mst}}
            print(f"[bench] {name} adjoint {msa:.4f} ms/step, from its tape {mst:.4f} ms/step",
                  file=sys.stderr, flush=True)
        adj["value"] = adj["f32"]["value"]
        adj["ms_per_step"] = adj["f32"]["ms_per_step"]

    # ---- full checkpointed backward pass over the workload's adjoint length
    backward = None
    SB = args.backward_steps if args.backward_steps >= 0 else (c.adjoint_steps or 0)
    if SB > 0:
        KB = c.ckpt_every or max(1, SB // 10)
        backward = {}
        for name, prec in (("f32", sg.FP32), ("f64", sg.FP64)):
            backward[name] = time_backward(torch, sg, c, prec, m0, alpha, SB, KB)
            torch.cuda.empty_cache()
            print(f"[bench] {name} backward pass, {SB} steps, checkpoints every {KB}: "
                  f"{backward[name]['backward_ms']:.1f} ms", file=sys.stderr, flush=True)

    # ---- the film workloads: one film-128x64 run (eager and graph-replayed steps) and
    # the adjoint film's checkpointed backward pass at its own length (500 steps,
    # checkpoints every 50)
    films = None
    if args.film_steps > 0:
        films = {}
        cf = workloads.config("film-128x64")
        pf = make_plan(sg, cf, sg.FP32)
        mf = torch.tensor(workloads.initial_state(cf), dtype=torch.float32, device="cuda")
        Bf = workloads.field_schedule(cf, 1)[0]
        pf.steps(mf, 10, cf.alpha, Bf)
        for _ in range(10):
            pf.step(mf, cf.alpha, Bf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.film_steps):
            pf.step(mf, cf.alpha, Bf)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pf.steps(mf, args.film_steps, cf.alpha, Bf)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pf.check()
        pf.close()
        ms_e, ms_g = (t1 - t0) * 1e3 / args.film_steps, (t2 - t1) * 1e3 / args.film_steps
        films["film-128x64"] = {"dtype": "f32", "steps": args.film_steps, "eager_ms_per_step": ms_e,
                                "graph_ms_per_step": ms_g, "value": cf.cells / (ms_g * 1e-3),
                                "unit": "cell-updates/s", "note": "value: graph-replayed steps (sgspm_steps)"}
        print(f"[bench] film-128x64 fp32 step: eager {ms_e:.4f} ms, graph-replayed {ms_g:.4f} ms",
              file=sys.stderr, flush=True)
        # many independent film runs in one batched plan (every launch covers all runs)
        BF = 64
        pb = make_plan(sg, cf, sg.FP32, batch=BF)
        m1 = torch.tensor(workloads.initial_state(cf), dtype=torch.float32, device="cuda")
        mb = m1.unsqueeze(1).expand(3, BF, *m1.shape[1:]).contiguous()
        alphas = [cf.alpha] * BF
        fields = [tuple(float(x) * (1.0 + 0.01 * b) for x in Bf) for b in range(BF)]
        pb.steps_batch(mb, 10, alphas, fields)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.steps_batch(mb, args.film_steps, alphas, fields)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3 / args.film_steps
        pb.check()
        pb.close()
        films["film-128x64_batched"] = {"dtype": "f32", "runs": BF, "steps": args.film_steps,
                                        "ms_per_step": ms_b, "value": BF * cf.cells / (ms_b * 1e-3),
                                        "unit": "cell-updates/s",
                                        "note": f"{BF} runs of the film (applied fields 1.00 to 1.63 times 5 mT) "
                                                "in one batched plan, graph-replayed batched steps"}
        print(f"[bench] film-128x64 x {BF} runs, batched: {ms_b:.4f} ms per step of all runs "
              f"({BF * cf.cells / (ms_b * 1e-3):.3e} cell-updates/s)", file=sys.stderr, flush=True)
        ca = workloads.config("adjoint-film-128x128")
        films["adjoint-film-128x128_backward"] = time_backward(
            torch, sg, ca, sg.FP32, workloads.initial_state(ca), ca.alpha, ca.adjoint_steps, ca.ckpt_every)
        print(f"[bench] adjoint-film-128x128 fp32 backward pass, {ca.adjoint_steps} steps, checkpoints every "
              f"{ca.ckpt_every}: {films['adjoint-film-128x128_backward']['backward_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    # ---- the strip workload as specified: 5 fields x 3 dampings, 15 independent runs,
    # FP64 energies every 10 steps (graph-replayed steps between the records)
    sweep = None
    if args.sweep_steps > 0:
        from paper_2606_28113_amd import runs as runs_mod
        cs = workloads.config("wall-strip-512x32x4")
        m0s = workloads.initial_state(cs)
        log = open(args.metrics_log, "w") if args.metrics_log else None
        cases = [(float(b_mT), a) for b_mT in cs.extra["fields_mT"] for a in cs.extra["alphas"]]
        t0 = time.perf_counter()
        # one batched plan: every launch of a step covers the 15 runs
        pb = make_plan(sg, cs, sg.FP32, batch=len(cases))
        mss = torch.tensor(np.repeat(m0s[:, None], len(cases), axis=1), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        r = runs_mod.run_batch(pb, mss, [a for _, a in cases], [(b * 1e-3, 0.0, 0.0) for b, _ in cases],
                               args.sweep_steps, log_every=10, sink=log, extras=[{"B_mT": b} for b, _ in cases])
        step_s = r["step_seconds"]
        detail = []
        for (b_mT, a), rec, mono in zip(cases, r["records"], r["monotone"]):
            detail.append({"B_mT": b_mT, "alpha": a, "monotone_energy": mono,
                           "E0": rec[0]["energy"]["total"], "E_end": rec[-1]["energy"]["total"],
                           "max_unit_error": max(x["unit_error"] for x in rec)})
        wall = time.perf_counter() - t0
        if log:
            log.close()
        pb.close()
        del mss
        cu = cs.cells * args.sweep_steps * len(detail)
        sweep = {"workload": f"{cs.name}: {WORKLOAD_TEXT[cs.name].split(', 5 mT')[0]}, fields "
                             f"{', '.join(f'{b:g}' for b in cs.extra['fields_mT'])} mT x alpha "
                             f"{', '.join(f'{a:g}' for a in cs.extra['alphas'])}, dt 0.1 ps",
                 "runs": len(detail), "steps_per_run": args.sweep_steps, "dtype": "f32",
                 "value": cu / step_s, "unit": "cell-updates/s", "step_seconds": step_s,
                 "value_incl_logging": cu / wall, "wall_s": wall,
                 "note": "15 runs in one batched plan (every launch of a step covers all runs; steps replayed "
                         "from a captured HIP graph of the batched step); FP64 energies per term of every run "
                         "and max ||m| - 1| over the runs every 10 steps (synchronising); value counts the "
                         "stepping alone",
                 "runs_with_monotone_energy": sum(1 for d in detail if d["monotone_energy"]),
                 "detail": detail}
        print(f"[bench] strip sweep: {len(detail)} runs x {args.sweep_steps} steps, stepping {step_s:.2f} s "
              f"({cu / step_s:.3e} cell-updates/s), wall {wall:.2f} s", file=sys.stderr, flush=True)

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
        "frozen_field": ff,
        "wall_sweep": sweep,
        "adjoint": adj,
        "backward_pass": backward,
        "films": films,
        "error_vs_oracle": err,
        "passes_ms_per_step": passes,
        "kernels": breakdown,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
