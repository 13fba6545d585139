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
