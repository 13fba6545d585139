"""GPU: graph-replayed stepping (sgspm_steps) against eager steps, the unit-length
error reduction, and the logged-run driver used by the strip workload's sweep."""
import numpy as np
import pytest

import workloads

from helpers import gpu_plan_si, to_dev

pytestmark = pytest.mark.gpu

ALL = ("exchange", "aniso", "stray", "zeeman")
CELL = (4e-9, 4e-9, 4e-9)
DT = 0.1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28113_amd as sg
    return torch, sg


@pytest.fixture(autouse=True)
def _announce(request):
    import sys
    sys.stderr.write(f"\n[gpu-case] {request.node.nodeid}\n")
    sys.stderr.flush()


@pytest.mark.parametrize("n,prec,scheme_", [((128, 64, 1), 0, 0), ((512, 32, 4), 0, 0), ((16, 256, 32), 1, 0),
                                            ((32, 16, 4), 0, 2), ((64, 32, 1), 1, 1)],
                         ids=["film-fp32", "strip-fp32", "block-fp64", "ff-fp32", "gspm-fp64"])
def test_graph_steps_match_eager(env, n, prec, scheme_):
    """Every replay of the captured step equals the eager steps bit for bit, with eager
    work on other arrays between the replays, and a new capture when alpha or h_e or
    the array change."""
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 400)
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec, scheme_=scheme_)
    ma, mb = to_dev(torch, m0, prec), to_dev(torch, m0, prec)
    other = to_dev(torch, workloads.random_unit(shape, 401), prec)
    B = (5e-3, 0.0, 1e-3)
    for rnd, (k, alpha, he) in enumerate([(4, 0.02, B), (3, 0.02, B), (2, 0.05, B), (3, 0.05, (0.0, 2e-3, 0.0))]):
        plan.steps(ma, k, alpha, he)
        for _ in range(k):
            plan.step(mb, alpha, he)
        plan.step(other, 0.01, (1e-3, 0.0, 0.0))  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(ma, mb), rnd
    # another array: captured again
    mc = to_dev(torch, m0, prec)
    plan.steps(mc, 2, 0.02, B)
    md = to_dev(torch, m0, prec)
    plan.step(md, 0.02, B)
    plan.step(md, 0.02, B)
    torch.cuda.synchronize()
    assert torch.equal(mc, md)
    plan.check()


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_unit_error(env, prec):
    torch, sg = env
    n = (64, 32, 2)
    m = workloads.random_unit((n[2], n[1], n[0]), 402)
    m[:, 1, 5, 7] *= 1.25
    m[:, 0, 0, 0] *= 0.5
    plan = gpu_plan_si(sg, n, CELL, DT, ("exchange",), prec)
    got = plan.unit_error(to_dev(torch, m, prec))
    mr = m.astype(np.float32).astype(np.float64) if prec == 0 else m
    ref = float(np.abs(np.sqrt(np.sum(mr * mr, axis=0)) - 1.0).max())
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_run_logged_strip(env):
    """The logged-run driver on the strip workload: records at step 0 and every 10 steps,
    energies equal to an eager run's, unit-length error at rounding level."""
    torch, sg = env
    from paper_2606_28113_amd import runs
    c = workloads.config("wall-strip-512x32x4")
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 0)
    m = to_dev(torch, workloads.initial_state(c), 0)
    sink = []
    out = runs.run_logged(plan, m, 40, 1e-3, (10e-3, 0.0, 0.0), log_every=10, sink=sink, run_id=3,
                          extra={"B_mT": 10.0})
    assert [r["step"] for r in out["records"]] == [0, 10, 20, 30, 40] and sink == out["records"]
    assert all(r["run"] == 3 and r["B_mT"] == 10.0 for r in sink)
    me = to_dev(torch, workloads.initial_state(c), 0)
    for _ in range(40):
        plan.step(me, 1e-3, (10e-3, 0.0, 0.0))
    e = plan.energy(me, (10e-3, 0.0, 0.0))
    assert e == out["records"][-1]["energy"]
    assert max(r["unit_error"] for r in sink) <= 1e-6
    E = [r["energy"]["total"] for r in sink]
    assert out["monotone"] == all(b <= a for a, b in zip(E, E[1:]))


def test_concurrent_sweep_matches_sequential_runs(env):
    """Runs stepped together on their own streams (run_sweep) give bit for bit the
    states and records of the same runs stepped one after another (run_logged)."""
    torch, sg = env
    from paper_2606_28113_amd import runs
    n = (128, 16, 2)
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 410)
    cases = [(0.01, (1e-3, 0.0, 0.0)), (0.001, (5e-3, 0.0, 0.0)), (0.0001, (2e-2, 0.0, 0.0)), (0.01, (0.0, 1e-2, 0.0))]
    plans, ms = [], []
    for _ in cases:
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            plans.append(gpu_plan_si(sg, n, CELL, DT, ALL, 0))
            ms.append(to_dev(torch, m0, 0))
    torch.cuda.synchronize()
    r = runs.run_sweep(plans, ms, [a for a, _ in cases], [b for _, b in cases], 25, log_every=10)
    ref_plan = gpu_plan_si(sg, n, CELL, DT, ALL, 0)
    for i, (a, b) in enumerate(cases):
        m = to_dev(torch, m0, 0)
        q = runs.run_logged(ref_plan, m, 25, a, b, log_every=10)
        torch.cuda.synchronize()
        assert torch.equal(m, ms[i]), i
        assert [x["step"] for x in r["records"][i]] == [0, 10, 20, 25]
        assert [x["energy"] for x in r["records"][i]] == [x["energy"] for x in q["records"]], i
        assert r["monotone"][i] == q["monotone"]
    for p in plans + [ref_plan]:
        p.close()
