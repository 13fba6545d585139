"""GPU: the allocation-free adjoint entry point (sgspm_adjoint_step_noalloc) against
the adjoint entry point it mirrors (sgspm_adjoint_step), on two calls in a row
whose second grid is smaller than the first, and its rejection of a grid beyond
its static workspace."""
import numpy as np
import pytest

import workloads
from oracle import adjoint as oadj

from helpers import gpu_plan_si, oracle_field_si, oracle_problem_si, to_dev

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


def _both(torch, sg, n, prec, seed):
    shape = (n[2], n[1], n[0])
    rng = np.random.default_rng(seed)
    m0 = workloads.random_unit(shape, seed + 1)
    lam = rng.normal(size=m0.shape)
    B = (4e-3, -1e-3, 2e-3)
    alpha = 0.03
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec)
    m_d = to_dev(torch, m0, prec)
    outs = []
    for fn in (plan.adjoint_step, plan.adjoint_step_noalloc):
        lam_d = to_dev(torch, lam, prec)
        grad = torch.zeros(4, dtype=torch.float64, device="cuda")
        fn(m_d, alpha, B, lam_d, grad)
        torch.cuda.synchronize()
        outs.append((lam_d.cpu().numpy(), grad.cpu().numpy()))
    return plan, m0, lam, B, alpha, outs


def test_noalloc_matches_adjoint_step_two_calls(env):
    torch, sg = env
    import sys
    # first call: the 128x128 film in single precision (16384 cells)
    sys.stderr.write("\n[gpu-case] noalloc call 1: 128x128x1 fp32\n")
    sys.stderr.flush()
    _, _, _, _, _, outs = _both(torch, sg, (128, 128, 1), 0, 300)
    (l_ref, g_ref), (l_na, g_na) = outs
    assert np.array_equal(l_na, l_ref)
    assert np.array_equal(g_na, g_ref)
    # second call, smaller grid, double precision: the workspace holds the first
    # call's values, which the second must not read
    sys.stderr.write("[gpu-case] noalloc call 2: 16x8x4 fp64\n")
    sys.stderr.flush()
    n = (16, 8, 4)
    _, m0, lam, B, alpha, outs = _both(torch, sg, n, 1, 310)
    (l_ref, g_ref), (l_na, g_na) = outs
    assert np.array_equal(l_na, l_ref)
    assert np.array_equal(g_na, g_ref)
    P = oracle_problem_si(n, CELL, DT, ALL)
    lref, dh, da = oadj.adjoint_step(P, m0, alpha, oracle_field_si(B, ALL), lam)
    assert np.abs(l_na - lref).max() <= 1e-11 * np.abs(lref).max()
    assert g_na[3] == pytest.approx(da, rel=1e-10, abs=1e-14)


def test_noalloc_rejects_grid_beyond_workspace(env):
    torch, sg = env
    # 256 x 256 x 4 = 262144 cells: 16 MiB of FP32 workspace, twice the static array
    n = (256, 256, 4)
    plan = gpu_plan_si(sg, n, CELL, DT, ("exchange",), 0)
    m = torch.zeros((3, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    m[2] = 1.0
    lam = torch.zeros_like(m)
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(sg.SGSPMError) as ei:
        plan.adjoint_step_noalloc(m, 0.01, (0.0, 0.0, 0.0), lam, grad)
    assert ei.value.code == sg.binding.EUNSUPPORTED
    assert "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert float(grad.abs().sum()) == 0.0
