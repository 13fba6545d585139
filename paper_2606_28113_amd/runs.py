"""Logged runs on one plan: constant (alpha, h_e) stepping by graph replay with
FP64 energies and the unit-length error recorded every few steps.

A record is one JSON object per line:
  {"run": id, "step": k, "alpha": a, "h_e": [..], "energy": {total, exchange,
   anisotropy, stray, zeeman}, "unit_error": max | |m| - 1 |, ...extra}
"""
import json
import time


def run_logged(plan, m, steps, alpha, h_e, log_every=10, sink=None, run_id=0, extra=None):
    """Advance m in place by `steps` steps of constant alpha and h_e (sgspm_steps), logging
    the energies and the unit-length error at step 0 and every `log_every` steps.

    sink: None, a list (records appended) or a text file (one JSON line per record).
    Returns {"records", "monotone" (total energy never rose between records),
    "step_seconds" (synchronised wall of the stepping alone), "seconds"}.
    """
    import torch
    records = []
    t_all = time.perf_counter()
    step_s = 0.0

    def record(k):
        e = plan.energy(m, h_e)
        r = {"run": run_id, "step": k, "alpha": alpha, "h_e": [float(x) for x in h_e], "energy": e,
             "unit_error": plan.unit_error(m)}
        if extra:
            r.update(extra)
        records.append(r)
        if sink is not None:
            if isinstance(sink, list):
                sink.append(r)
            else:
                sink.write(json.dumps(r) + "\n")

    record(0)
    done = 0
    while done < steps:
        k = min(log_every, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.steps(m, k, alpha, h_e)
        torch.cuda.synchronize()
        step_s += time.perf_counter() - t0
        done += k
        record(done)
    plan.check()
    E = [r["energy"]["total"] for r in records]
    mono = all(b <= a for a, b in zip(E, E[1:]))
    return {"records": records, "monotone": mono, "step_seconds": step_s,
            "seconds": time.perf_counter() - t_all}


def run_sweep(plans, ms, alphas, fields, steps, log_every=10, sink=None, extras=None):
    """Advance independent runs together, each on its own plan and HIP stream.

    plans[i] must have been created under a stream of its own (torch.cuda.stream),
    with ms[i] allocated under the same stream; every run steps with constant
    alphas[i] and fields[i] by graph replay on its plan's stream, so the small
    launches of different runs execute concurrently.  After every `log_every`
    steps of all runs the device is synchronised and each run's energies and
    unit-length error are recorded as in run_logged (run id i, plus extras[i]).

    Returns {"records": per-run lists, "monotone": per-run bools, "step_seconds"
    (synchronised wall of the stepping alone), "seconds"}.
    """
    import torch
    n = len(plans)
    records = [[] for _ in range(n)]
    t_all = time.perf_counter()
    step_s = 0.0

    def record(i, k):
        p, m = plans[i], ms[i]
        with torch.cuda.stream(p.stream):
            r = {"run": i, "step": k, "alpha": alphas[i], "h_e": [float(x) for x in fields[i]],
                 "energy": p.energy(m, fields[i]), "unit_error": p.unit_error(m)}
        if extras:
            r.update(extras[i])
        records[i].append(r)
        if sink is not None:
            if isinstance(sink, list):
                sink.append(r)
            else:
                sink.write(json.dumps(r) + "\n")

    for i in range(n):
        record(i, 0)
    done = 0
    while done < steps:
        k = min(log_every, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            with torch.cuda.stream(plans[i].stream):
                plans[i].steps(ms[i], k, alphas[i], fields[i])
        torch.cuda.synchronize()
        step_s += time.perf_counter() - t0
        done += k
        for i in range(n):
            record(i, done)
    for p in plans:
        p.check()
    mono = [all(b["energy"]["total"] <= a["energy"]["total"] for a, b in zip(rs, rs[1:])) for rs in records]
    return {"records": records, "monotone": mono, "step_seconds": step_s, "seconds": time.perf_counter() - t_all}


def run_batch(plan, m, alphas, fields, steps, log_every=10, sink=None, extras=None):
    """Advance the runs of a batched plan together (sgspm_steps_batch: every launch of
    a step covers all runs), recording every run's energies every `log_every` steps
    as run_logged does; "unit_error" is the maximum over all runs of the batch.

    m: (3, B, nz, ny, nx); alphas: B values; fields: B applied fields (3 each).
    Returns {"records": per-run lists, "monotone": per-run bools, "step_seconds",
    "seconds"}.
    """
    import torch
    B = plan.batch
    records = [[] for _ in range(B)]
    t_all = time.perf_counter()
    step_s = 0.0

    def record(k):
        es = plan.energy_batch(m, fields)
        ue = plan.unit_error(m)
        for i in range(B):
            r = {"run": i, "step": k, "alpha": alphas[i], "h_e": [float(x) for x in fields[i]], "energy": es[i],
                 "unit_error": ue}
            if extras:
                r.update(extras[i])
            records[i].append(r)
            if sink is not None:
                if isinstance(sink, list):
                    sink.append(r)
                else:
                    sink.write(json.dumps(r) + "\n")

    record(0)
    done = 0
    while done < steps:
        k = min(log_every, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.steps_batch(m, k, alphas, fields)
        torch.cuda.synchronize()
        step_s += time.perf_counter() - t0
        done += k
        record(done)
    plan.check()
    mono = [all(b["energy"]["total"] <= a["energy"]["total"] for a, b in zip(rs, rs[1:])) for rs in records]
    return {"records": records, "monotone": mono, "step_seconds": step_s, "seconds": time.perf_counter() - t_all}
