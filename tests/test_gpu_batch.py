"""GPU: batched plans, whose independent runs share every launch of a step.  Each
run of a batch equals, bit for bit, the same run on its own single-run plan
(states after several steps and FP64 energies); graph-replayed batched steps
equal the eager ones."""
import numpy as np
import pytest

import workloads

from helpers import gpu_plan_si, term_mask, to_dev

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


def _batched_plan(sg, n, prec, B, scheme_=0):
    return sg.Plan(nx=n[0], ny=n[1], nz=n[2], dx=CELL[0], dy=CELL[1], dz=CELL[2], dt=DT, units=sg.UNITS_SI,
                   A=workloads.A_PY, Ms=workloads.MS_PY, Ku=workloads.K_PY, terms=term_mask(ALL), precision=prec,
                   scheme=scheme_, batch=B)


def _runs(B):
    alphas = [0.02 * (1 + 0.5 * b) for b in range(B)]
    fields = [(5e-3 * (1 + b), 1e-3 * (b - 1), -2e-3) for b in range(B)]
    return alphas, fields


# the strip (generic row kernels, y pass, 8-point z convolution), a film (no y
# pass: the convolution runs along y), rows of 256 (register row kernels) with
# the 64-point convolution, and the 256 x 32 register y-z planes with the 512-point
# y pass and the packed DC / Nyquist layout; a mixed-radix grid
CASES = [((512, 32, 4), 0, 3, 0), ((128, 64, 1), 1, 2, 1), ((256, 8, 32), 0, 2, 0), ((16, 256, 32), 0, 2, 0),
         ((16, 256, 32), 1, 2, 0), ((100, 20, 4), 0, 2, 0)]


@pytest.mark.parametrize("n,prec,B,scheme_", CASES,
                         ids=["strip-fp32-B3", "film-fp64-B2-gspm", "256x8x32-fp32-B2", "16x256x32-fp32-B2",
                              "16x256x32-fp64-B2", "100x20x4-fp32-B2"])
def test_batched_runs_equal_single_runs(env, n, prec, B, scheme_):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = np.stack([workloads.random_unit(shape, 500 + b) for b in range(B)], axis=1)  # (3, B, nz, ny, nx)
    alphas, fields = _runs(B)
    plan = _batched_plan(sg, n, prec, B, scheme_)
    m = to_dev(torch, m0, prec)
    # energies before any batched step (the per-run values are not set yet)
    e0 = plan.energy_batch(m, fields)
    for _ in range(4):
        plan.step_batch(m, alphas, fields)
    torch.cuda.synchronize()
    plan.check()
    eb = plan.energy_batch(m, fields)
    for b in range(B):
        p1 = gpu_plan_si(sg, n, CELL, DT, ALL, prec, scheme_=scheme_)
        mb = to_dev(torch, np.ascontiguousarray(m0[:, b]), prec)
        assert e0[b] == p1.energy(mb, fields[b]), b
        for _ in range(4):
            p1.step(mb, alphas[b], fields[b])
        torch.cuda.synchronize()
        assert torch.equal(m[:, b], mb), b
        assert eb[b] == p1.energy(mb, fields[b]), b
        p1.close()
    plan.close()


@pytest.mark.parametrize("n,prec", [((512, 32, 4), 0), ((16, 256, 32), 0)], ids=["strip-fp32", "16x256x32-fp32"])
def test_batched_graph_steps_equal_eager(env, n, prec):
    """Replays of the captured batched step equal eager batched steps bit for bit,
    also after the per-run values change (read from the plan's buffer at replay)."""
    torch, sg = env
    B = 3
    shape = (n[2], n[1], n[0])
    m0 = np.stack([workloads.random_unit(shape, 520 + b) for b in range(B)], axis=1)
    plan = _batched_plan(sg, n, prec, B)
    ma, mb = to_dev(torch, m0, prec), to_dev(torch, m0, prec)
    alphas, fields = _runs(B)
    for rnd, (k, a, f) in enumerate([(3, alphas, fields), (2, alphas[::-1], fields),
                                     (2, alphas, [(0.0, 2e-3, 0.0)] * B)]):
        plan.steps_batch(ma, k, a, f)
        for _ in range(k):
            plan.step_batch(mb, a, f)
        torch.cuda.synchronize()
        assert torch.equal(ma, mb), rnd
    plan.close()


def test_batched_plan_rejects_single_run_calls(env):
    torch, sg = env
    plan = _batched_plan(sg, (16, 8, 4), 0, 2)
    m = torch.zeros(plan.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(sg.SGSPMError):
        plan.energy(m, (0.0, 0.0, 0.0))
    with pytest.raises(ValueError):
        plan.step_batch(m, [0.01], [(0.0, 0.0, 0.0)])
    plan.close()
