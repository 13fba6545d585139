"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle,
element by element, on the same seeded inputs.

Tolerances: FP64 plans agree with the oracle to rounding (1e-12 relative on
the linear operators; the stray field to the classical FFT rounding bound once
the measured difference of the two FP64 Newell tensors is taken out, and that
difference entry by entry to a bound pinned on the CPU); FP32 plans to a few FP32 ulps scaled
by the transform depth (5e-6 relative on linear operators), and to 1e-5 max-abs
in m after 1000 steps of the 128x64 film (the stated target).
"""
import functools

import numpy as np
import pytest
from scipy import fft as sfft

import newell_bounds as nb

import workloads
from oracle import demag, manufactured as mf, operators, scheme, spectral

from helpers import (gpu_plan_reduced, gpu_plan_si, oracle_field_si, oracle_problem_si, rounded_like,
                     to_dev)

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


HEAT_SHAPES = [(32, 32, 1), (128, 64, 1), (16, 8, 4), (8, 1, 1), (1, 1, 1), (1, 16, 1), (4, 1, 8),
               (64, 32, 8), (2, 2, 2), (512, 32, 4), (1024, 2, 1), (256, 256, 32), (8, 256, 32)]


@pytest.mark.parametrize("n", HEAT_SHAPES, ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_heat_solve(env, n, prec):
    torch, sg = env
    rng = np.random.default_rng(100)
    shape = (n[2], n[1], n[0])
    h = tuple(1.0 / k if k > 1 else 1.0 for k in n)
    plan = gpu_plan_reduced(sg, n, h, 0.01, 1.0, 0.0, ("exchange",), prec)
    r = rng.normal(size=shape)
    for s in (1.0, 0.37, 0.0):
        g = plan.heat_solve(to_dev(torch, r, prec), s).cpu().numpy()
        ref = operators.heat_solve(rounded_like(r, prec), s * 1.0 * 0.01, h)
        tol = 1e-12 if prec == 1 else 5e-6
        assert np.abs(g - ref).max() <= tol * np.abs(r).max(), (n, s)
        if s == 0.0:
            # the correction form: a zero diagonal leaves the right-hand side untouched
            assert np.array_equal(g, rounded_like(r, prec)), n


@pytest.mark.parametrize("n", [(128, 128, 1), (512, 32, 4), (256, 256, 32)], ids=lambda v: "x".join(map(str, v)))
def test_repeated_heat_solves_keep_their_scale(env, n):
    """50 FP32 heat solves in a row, each on the previous one's output, against the
    oracle's 50 exact solves from the same rounded start: a smooth field and white noise,
    at the damping scale (s = alpha = 0.01, x ~ 2e-7 k^2 in SI workload units) and the
    precession scale (s = 1). Storing each result in FP32 loses every change below half
    an ulp, so even exact solves rounded to FP32 after each one (the storage model)
    drift from the exact result; the scale the library keeps, <e, g> / <g, g> with
    e = g_lib - g_exact, must agree with the storage model's to 3e-7. A transform pair
    that lost 1e-7 of its input per solve (FP32 twiddles with c^2 + s^2 < 1) is 5e-6
    off after the 50 solves. Max-abs error within 3e-6 of max |g|."""
    torch, sg = env
    shape = (n[2], n[1], n[0])
    plan = gpu_plan_si(sg, n, CELL, DT, ("exchange",), 0)
    P = oracle_problem_si(n, CELL, DT, ("exchange",))
    z, y, x = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    smooth = 0.3 + np.cos(np.pi * (x + 0.5) / n[0]) * np.cos(np.pi * (y + 0.5) / n[1]) + 0.2 * np.sin(2 * np.pi * x / n[0])
    noise = np.random.default_rng(7).standard_normal(shape)

    def scale(g, ref):
        return float(((g - ref) * ref).sum() / (ref * ref).sum())

    for lab, f in (("smooth", smooth), ("noise", noise)):
        for s in (0.01, 1.0):
            r0 = rounded_like(f, 0)
            g = to_dev(torch, r0, 0)
            ex, st = r0.copy(), r0.copy()
            for _ in range(50):
                g = plan.heat_solve(g, s)
                ex = operators.heat_solve(ex, s * P.eps_eff * P.dt, P.h)
                st = rounded_like(operators.heat_solve(st, s * P.eps_eff * P.dt, P.h), 0)
            G = g.double().cpu().numpy()
            k_lib, k_st = scale(G, ex), scale(st, ex)
            err = float(np.abs(G - ex).max() / np.abs(ex).max())
            print(f"{'x'.join(map(str, n))} {lab} s={s}: 50 FP32 solves, scale vs exact {k_lib:+.1e} "
                  f"(storage model {k_st:+.1e}), max err {err:.1e}")
            assert abs(k_lib - k_st) <= 3e-7 and err <= 3e-6, (lab, s, k_lib, k_st, err)


# (16|32|256, 256, 32) pack the real DC and Nyquist x bins into bin 0 and keep the
# y-level Nyquist column in the blocked layout; (8, 256, 32) runs the same
# 512-point y pass and 64-point convolution without that packing (nx not a
# multiple of 16)
STRAY_SHAPES = [(8, 4, 2), (16, 8, 1), (4, 4, 4), (32, 1, 1), (1, 1, 1), (2, 2, 2), (1, 8, 4), (4, 1, 4),
                (128, 64, 1), (64, 32, 8), (512, 32, 4), (128, 128, 1), (16, 8, 32), (16, 32, 1), (4, 1, 32),
                (256, 4, 32), (16, 256, 2), (8, 256, 4), (32, 256, 32), (8, 2, 32), (16, 256, 32),
                (256, 256, 32), (8, 256, 32), (256, 256, 1), (256, 128, 1)]


@functools.lru_cache(maxsize=2)
def _spectra(shape):
    # the FP64 Newell spectra of the oracle (about 30 s at 256x256x32), shared by both precisions
    return demag.kernel_spectra(shape, CELL)


@functools.lru_cache(maxsize=1)
def _padded(shape, h):
    return nb.padded_tensor(shape, h)


@pytest.mark.parametrize("n,h", [((8, 4, 2), CELL), ((16, 8, 4), (4e-9, 4e-9, 2e-9)), ((64, 32, 8), CELL),
                                 ((32, 1, 1), CELL), ((256, 256, 32), CELL)],
                         ids=lambda v: "x".join(map(str, v)) if isinstance(v[0], int) else "x".join(f"{x:g}" for x in v))
def test_demag_tensor(env, n, h):
    """The FP64 demagnetising tensor the plan builds, entry by entry against the oracle's,
    within the per-entry rounding bound of two FP64 evaluations (2 KAPPA u S(d) for the
    Newell sums, which cancel, KAPPA pinned on the CPU; 8 u |N| for the dipole form)."""
    torch, sg = env
    shape = (n[2], n[1], n[0])
    plan = gpu_plan_si(sg, n, h, DT, ALL, 1)
    No, offs = nb.padded_tensor(shape, h)
    bound = nb.entry_bound(shape, h, No, offs)
    worst = 0.0
    for k, c in enumerate(demag.COMPONENTS):
        Ng = plan.demag_tensor(k).cpu().numpy()
        d = np.abs(Ng - No[c])
        assert np.all(d <= bound[c]), (c, float(d.max()))
        worst = max(worst, float((d / np.where(bound[c] > 0, bound[c], 1.0)).max()))
    print(f"demag tensor {n} cell {h}: max |N_gpu - N_oracle| / bound = {worst:.3f}")


@pytest.mark.parametrize("n", STRAY_SHAPES, ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_stray_field(env, n, prec):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m = workloads.random_unit(shape, 101)
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec)
    hs = plan.stray(to_dev(torch, m, prec)).cpu().numpy()
    ref = demag.stray_field(rounded_like(m, prec), _spectra(shape))
    err = np.abs(hs - ref).max()
    if prec == 0:
        print(f"stray fp32 {n}: max abs err {err:.3e} (bar 2e-6)")
        assert err <= 2e-6
        return
    # FP64: the library's tensor and the oracle's differ by the rounding of their
    # Newell sums (test_demag_tensor bounds it entry by entry).  That difference is
    # measured here and its field, -(N_gpu - N_oracle) (*) m, taken out exactly; what
    # remains is the two FFT convolutions' rounding, held to its classical bound.
    No, _ = _padded(shape, CELL)
    Pp = demag.padded_shape(shape)
    dN = {c: plan.demag_tensor(k).cpu().numpy() - No[c] for k, c in enumerate(demag.COMPONENTS)}
    dh = demag.stray_field(m, (Pp, {c: sfft.rfftn(dN[c]) for c in dN}))
    resid = np.abs(hs - ref - dh).max()
    fb = nb.fft_conv_bound(shape, _spectra(shape), m)
    # worst case over every field with |m_b| <= 1 of the tensor difference's field
    tens = max(sum(float(np.abs(dN[demag._PAIR[(a, b)]]).sum()) for b in range(3)) for a in range(3))
    print(f"stray fp64 {n}: max abs err {err:.3e} (bound sum|dN| + fft {tens + fb:.2e}); "
          f"after removing the tensor difference {resid:.3e} (fft bound {fb:.1e}, ratio {resid / fb:.2f})")
    assert resid <= fb
    assert err <= tens + fb


@pytest.mark.parametrize("n", [(16, 8, 4), (32, 32, 1), (64, 1, 1), (8, 8, 8), (16, 256, 32)],
                         ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_effective_field_and_energy(env, n, prec):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m = workloads.random_unit(shape, 102)
    B = (3e-3, -1e-3, 2e-3)
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec)
    P = oracle_problem_si(n, CELL, DT, ALL)
    he = oracle_field_si(B, ALL)
    md = to_dev(torch, m, prec)
    h = plan.field(md, B).cpu().numpy()
    m64 = rounded_like(m, prec)
    ref = scheme.effective_field(P, m64, he)
    scale = np.abs(ref).max()
    err = np.abs(h - ref).max()
    e = plan.energy(md, B)
    eref = scheme.energies(P, m64, he)
    mu0ms2 = 4e-7 * np.pi * workloads.MS_PY ** 2
    erel = {k: abs(e[k] / mu0ms2 - eref[k]) / (abs(eref["total"]) + abs(eref[k]) + 1e-30) for k in eref}
    print(f"field {'fp64' if prec else 'fp32'} {n}: max err / scale {err / scale:.2e}; energies "
          + ", ".join(f"{k} {v:.1e}" for k, v in erel.items()))
    assert err <= (1e-11 if prec == 1 else 3e-6) * scale
    for k in eref:
        assert erel[k] <= (1e-11 if prec == 1 else 1e-6), k


def _run_gpu(plan, torch, m0, alphas, fields, prec, src=None):
    m = to_dev(torch, m0, prec)
    for n in range(len(fields)):
        plan.step(m, alphas[n] if np.ndim(alphas) else alphas, fields[n],
                  None if src is None else to_dev(torch, src[n], prec))
    torch.cuda.synchronize()
    plan.check()
    return m.cpu().numpy()


SCHEME = {"sgspm": 0, "gspm": 1, "sgspm_ff": 2}


def _run_oracle(P, m0, alpha, fields, method="sgspm", src=None):
    step = {"sgspm": scheme.sgspm_step, "gspm": scheme.gspm_step, "sgspm_ff": scheme.sgspm_ff_step}[method]
    m = np.asarray(m0, np.float64)
    for n in range(len(fields)):
        m = step(P, m, alpha, fields[n], src=None if src is None else src[n])
    return m


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_manufactured_film_32x32(env, prec):
    """32x32 exchange-only film with the 2-D manufactured forcing, 200 steps."""
    torch, sg = env
    c = workloads.config("mf-film-32x32")
    shape = c.shape
    plan = gpu_plan_reduced(sg, c.n, c.h, c.dt, c.eps, 0.0, ("exchange",), prec)
    m0 = workloads.initial_state(c)
    src = [mf.forcing(shape, k * c.dt, 2, c.eps, c.alpha) for k in range(c.steps)]
    fields = [(0.0, 0.0, 0.0)] * c.steps
    got = _run_gpu(plan, torch, m0, c.alpha, fields, prec, src=src)
    P = scheme.Problem(n=c.n, h=c.h, eps=c.eps, dt=c.dt)
    src64 = [rounded_like(s, prec) for s in src]
    ref = _run_oracle(P, rounded_like(m0, prec), c.alpha, fields, src=src64)
    err = np.abs(got - ref).max()
    print(f"mf-film {'fp64' if prec else 'fp32'}: max|m - m_oracle| = {err:.3e}; "
          f"max|m - m_exact| = {np.abs(got - mf.exact(shape, c.steps * c.dt, 2)).max():.3e}")
    assert err <= (1e-11 if prec == 1 else 1e-5)


@pytest.mark.parametrize("n", [(16, 8, 4), (32, 16, 1), (8, 1, 8), (16, 1, 1), (256, 4, 2), (256, 1, 1)],
                         ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("method", ["sgspm", "gspm", "sgspm_ff"])
def test_full_step_fp64(env, n, method):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 103)
    B = [(5e-3, 1e-3, -2e-3)] * 10
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, 1, scheme_=SCHEME[method])
    got = _run_gpu(plan, torch, m0, 0.02, B, 1)
    P = oracle_problem_si(n, CELL, DT, ALL)
    ref = _run_oracle(P, m0, 0.02, [oracle_field_si(b, ALL) for b in B], method)
    assert np.abs(got - ref).max() <= 1e-10


# rows of 256 (the 512-point row kernels), the 512-point y pass with and without
# the DC/Nyquist packing, the 64-point convolution and the 256x32 register y-z
# solve, through whole steps from a random start; rows of 256 in odd number
# (3, 15), whose x-major heat arrays the register row kernels cannot pair, run the
# generic row kernels
@pytest.mark.parametrize("n", [(16, 256, 32), (256, 256, 1), (256, 8, 32), (256, 3, 1), (256, 5, 3)],
                         ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_steps_512_paths(env, n, prec):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 106)
    B = [(5e-3, 1e-3, -2e-3)] * 5
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec)
    got = _run_gpu(plan, torch, m0, 0.02, B, prec)
    P = oracle_problem_si(n, CELL, DT, ALL)
    ref = _run_oracle(P, rounded_like(m0, prec), 0.02, [oracle_field_si(b, ALL) for b in B])
    err = np.abs(got - ref).max()
    print(f"steps {'fp64' if prec else 'fp32'} {n}: max|m - m_oracle| after 5 steps = {err:.3e}")
    assert err <= (1e-10 if prec == 1 else 1e-5)


@pytest.mark.parametrize("terms", [("exchange",), ("exchange", "aniso"), ("stray",), ("exchange", "zeeman"),
                                   ("aniso", "stray", "zeeman")], ids=lambda t: "+".join(t))
def test_term_subsets_fp64(env, terms):
    torch, sg = env
    n = (16, 8, 2)
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 104)
    B = [(5e-3, 1e-3, -2e-3)] * 5
    plan = gpu_plan_si(sg, n, CELL, DT, terms, 1)
    got = _run_gpu(plan, torch, m0, 0.05, B, 1)
    P = oracle_problem_si(n, CELL, DT, terms)
    ref = _run_oracle(P, m0, 0.05, [oracle_field_si(b, terms) for b in B])
    assert np.abs(got - ref).max() <= 1e-10


def test_film_128x64_fp64_random_start(env):
    """128x64 permalloy-like film, all fields, 5 mT, alpha 0.01, from i.i.d. random unit vectors:
    the FP64 library against the FP64 oracle.

    This start is chaotic: two oracle runs whose m0 differ by 1e-7 drift apart to 5e-6 after
    100 steps, 6e-5 after 200 and O(1) after 700.  The two FP64 implementations differ by
    ~1e-12 per Newell-tensor entry (independent libm, cancellation), which that growth lifts to
    ~1e-4 by step 1000; the test bounds the early steps and sanity-checks step 1000."""
    torch, sg = env
    c = workloads.config("film-128x64")
    m0 = workloads.initial_state(c)
    B = workloads.field_schedule(c)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 1)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    m = to_dev(torch, m0, 1)
    ref = np.asarray(m0, np.float64)
    done = 0
    for k, tol in ((100, 2e-8), (200, 1e-7), (1000, 1e-2)):
        for n in range(done, k):
            plan.step(m, c.alpha, B[n])
            ref = scheme.sgspm_step(P, ref, c.alpha, oracle_field_si(B[n], ALL))
        done = k
        err = np.abs(m.cpu().numpy() - ref).max()
        print(f"film-128x64 fp64 random start, step {k}: max|m - m_oracle| = {err:.3e}")
        assert err <= tol, k


def test_film_128x64_fp32_random_start_early(env):
    """FP32 on the chaotic random start of the 128x64 film: bounded while the trajectory sensitivity is moderate."""
    torch, sg = env
    c = workloads.config("film-128x64")
    m0 = workloads.initial_state(c)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 0)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    he = oracle_field_si((5e-3, 0.0, 0.0), ALL)
    m = to_dev(torch, m0, 0)
    ref = rounded_like(m0, 0)
    done = 0
    for k, tol in ((1, 1e-6), (10, 1e-5), (100, 2e-4)):
        for _ in range(k - done):
            plan.step(m, c.alpha, (5e-3, 0.0, 0.0))
            ref = scheme.sgspm_step(P, ref, c.alpha, he)
        done = k
        err = np.abs(m.cpu().numpy() - ref).max()
        print(f"film-128x64 fp32 random start, step {k}: max|m - m_oracle| = {err:.3e}")
        assert err <= tol, k


def test_film_128x64_fp32_1000_steps_paper_start(env):
    """128x64 film, all fields, 1000 steps from the paper's eq. (m0-1) state, a well-conditioned
    trajectory (a 1e-7 perturbation stays below 4e-7): FP32 library within 1e-5 of the FP64 oracle."""
    torch, sg = env
    c = workloads.config("film-128x64")
    m0 = workloads.paper_ic(c.shape)
    B = workloads.field_schedule(c)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 0)
    got = _run_gpu(plan, torch, m0, c.alpha, B, 0)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    ref = _run_oracle(P, rounded_like(m0, 0), c.alpha, [oracle_field_si(b, ALL) for b in B])
    err = np.abs(got - ref).max()
    e_gpu = plan.energy(to_dev(torch, got, 0), B[-1])["total"]
    e_ref = scheme.energies(P, ref, oracle_field_si(B[-1], ALL))["total"] * 4e-7 * np.pi * workloads.MS_PY ** 2
    print(f"film-128x64 fp32 1000 steps (paper start): max|m - m_oracle| = {err:.3e}, "
          f"relative energy error {abs(e_gpu - e_ref) / abs(e_ref):.3e}")
    assert err <= 1e-5


def test_wall_strip_512x32x4_fp64_20_steps(env):
    torch, sg = env
    c = workloads.config("wall-strip-512x32x4")
    m0 = workloads.initial_state(c)
    B = [(10e-3, 0.0, 0.0)] * 20
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 1)
    got = _run_gpu(plan, torch, m0, 1e-3, B, 1)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    ref = _run_oracle(P, m0, 1e-3, [oracle_field_si(b, ALL) for b in B])
    assert np.abs(got - ref).max() <= 1e-10


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_block_256x256x32_one_step(env, prec):
    """256x256x32 block, full fields, one step at full size (the benchmark launch shapes)."""
    torch, sg = env
    c = workloads.config("block-256x256x32")
    m0 = workloads.initial_state(c)
    B = workloads.field_schedule(c, 1)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, prec)
    got = _run_gpu(plan, torch, m0, c.alpha, B, prec)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    ref = _run_oracle(P, rounded_like(m0, prec), c.alpha, [oracle_field_si(b, ALL) for b in B])
    err = np.abs(got - ref).max()
    print(f"block {'fp64' if prec else 'fp32'} one step: max|m - m_oracle| = {err:.3e}")
    assert err <= (1e-10 if prec == 1 else 2e-6)


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_wall_strip_512x32x4_50_steps(env, prec):
    """The strip workload's grid and Neel-wall start, all fields, 50 steps at its stated
    alpha and field, in both precisions against the FP64 oracle (FP32 from FP32-rounded inputs)."""
    torch, sg = env
    c = workloads.config("wall-strip-512x32x4")
    m0 = workloads.initial_state(c)
    B = workloads.field_schedule(c, 50)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, prec)
    got = _run_gpu(plan, torch, m0, c.alpha, B, prec)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    ref = _run_oracle(P, rounded_like(m0, prec), c.alpha, [oracle_field_si(b, ALL) for b in B])
    err = np.abs(got - ref).max()
    print(f"wall-strip {'fp64' if prec else 'fp32'} 50 steps: max|m - m_oracle| = {err:.3e}")
    assert err <= (1e-10 if prec == 1 else 1e-5)


# GSPM (paper §3.1) in single precision, on the generic kernels and on the
# 512-point / register paths of the block
@pytest.mark.parametrize("n", [(16, 8, 4), (32, 16, 1), (256, 4, 2), (16, 256, 32)],
                         ids=lambda n: "x".join(map(str, n)))
def test_gspm_fp32(env, n):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.paper_ic(shape)
    B = [(5e-3, 1e-3, -2e-3)] * 10
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, 0, scheme_=1)
    got = _run_gpu(plan, torch, m0, 0.02, B, 0)
    P = oracle_problem_si(n, CELL, DT, ALL)
    ref = _run_oracle(P, rounded_like(m0, 0), 0.02, [oracle_field_si(b, ALL) for b in B], "gspm")
    err = np.abs(got - ref).max()
    print(f"gspm fp32 {n}: max|m - m_oracle| after 10 steps = {err:.3e}")
    assert err <= 1e-5


# the frozen-field reading (two stray-field evaluations per step) on the generic
# kernels, the 512-point / register paths, and at the benchmark's full size
@pytest.mark.parametrize("n", [(16, 8, 4), (128, 64, 1), (16, 256, 32), (256, 256, 32)],
                         ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_sgspm_ff_steps(env, n, prec):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 107) if n[0] * n[1] * n[2] < 1 << 20 else workloads.box_smoothed_unit(shape, 5)
    steps = 5 if n[0] * n[1] * n[2] < 1 << 20 else 1
    B = [(5e-3, 1e-3, -2e-3)] * steps
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec, scheme_=2)
    got = _run_gpu(plan, torch, m0, 0.02, B, prec)
    P = oracle_problem_si(n, CELL, DT, ALL)
    ref = _run_oracle(P, rounded_like(m0, prec), 0.02, [oracle_field_si(b, ALL) for b in B], "sgspm_ff")
    err = np.abs(got - ref).max()
    print(f"sgspm-ff {'fp64' if prec else 'fp32'} {n}: max|m - m_oracle| after {steps} steps = {err:.3e}")
    assert err <= (1e-10 if prec == 1 else 1e-5)


# spectral radius of the sweep matrices (§4) per step, against the oracle's per-cell
# eigenvalues, and the step it rides on
@pytest.mark.parametrize("n", [(16, 8, 4), (128, 64, 1), (16, 256, 32)], ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_spectral_radius(env, n, prec):
    torch, sg = env
    shape = (n[2], n[1], n[0])
    m0 = workloads.random_unit(shape, 108)
    B = (5e-3, 1e-3, -2e-3)
    P = oracle_problem_si(n, CELL, DT, ALL)
    ref = spectral.spectral_radii(P, rounded_like(m0, prec), 0.02, oracle_field_si(B, ALL))
    m_ref = scheme.sgspm_step(P, rounded_like(m0, prec), 0.02, oracle_field_si(B, ALL))
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, prec)
    m = to_dev(torch, m0, prec)
    r = plan.step_spectral_radius(m, 0.02, B)
    e = [abs(r[k] - ref[k]) / ref[k] for k in range(2)]
    print(f"spectral radius {'fp64' if prec else 'fp32'} {n}: GS {r[0]:.6e} (oracle {ref[0]:.6e}), "
          f"SGS {r[1]:.6e} (oracle {ref[1]:.6e}); rel err {e[0]:.1e}, {e[1]:.1e}")
    bar = 1e-9 if prec == 1 else 1e-5
    assert max(e) <= bar
    assert np.abs(m.cpu().numpy() - m_ref).max() <= (1e-10 if prec == 1 else 2e-6)
    # a GSPM plan reports the forward sweep's radius only
    gp = gpu_plan_si(sg, n, CELL, DT, ALL, prec, scheme_=1)
    rg = gp.step_spectral_radius(to_dev(torch, m0, prec), 0.02, B)
    assert np.isnan(rg[1]) and abs(rg[0] - ref[0]) / ref[0] <= bar


@pytest.mark.parametrize("dim", [1, 3])
def test_energy_decay_sgspm_vs_gspm(env, dim):
    """The paper's central comparison (§3.1 and §3.2 energy figures, §5.2) on the GPU:
    exchange only (eps = 1), from eq. (m0-1), FP64, 60 steps of dt = 0.01.  SGSPM's
    energy falls at every step for every alpha in {0, 0.005, 0.01, 0.1, 0.5}; GSPM's
    rises at some step for alpha in {0, 0.005, 0.01} and falls for 0.1 and 0.5.  Every
    energy also matches the oracle's along its own trajectory."""
    torch, sg = env
    n = (64, 1, 1) if dim == 1 else (16, 16, 16)
    shape = (n[2], n[1], n[0])
    h = tuple(1.0 / k if k > 1 else 1.0 for k in n)
    P = scheme.Problem(n=n, h=h, eps=1.0, dt=0.01)
    steps = 60
    worst = 0.0
    for method, alphas in (("sgspm", (0.0, 0.005, 0.01, 0.1, 0.5)), ("gspm", (0.0, 0.005, 0.01, 0.1, 0.5))):
        plan = gpu_plan_reduced(sg, n, h, 0.01, 1.0, 0.0, ("exchange",), 1, scheme_=SCHEME[method])
        ostep = scheme.sgspm_step if method == "sgspm" else scheme.gspm_step
        for alpha in alphas:
            m = to_dev(torch, workloads.paper_ic(shape), 1)
            ref = workloads.paper_ic(shape)
            E = [plan.energy(m, (0, 0, 0))["total"]]
            for _ in range(steps):
                plan.step(m, alpha, (0.0, 0.0, 0.0))
                ref = ostep(P, ref, alpha, (0, 0, 0))
                E.append(plan.energy(m, (0, 0, 0))["total"])
                er = scheme.energies(P, ref, (0, 0, 0))["total"]
                worst = max(worst, abs(E[-1] - er) / abs(er))
            dE = np.diff(E)
            print(f"{dim}-D {method} alpha {alpha}: E0 {E[0]:.6e}, E_end {E[-1]:.6e}, max step change {dE.max():+.3e}")
            if method == "sgspm" or alpha >= 0.1:
                assert np.all(dE < 0), (method, alpha)
            else:
                # GSPM's energy rises for alpha <= 0.01 on this start (the oracle agrees)
                assert dE.max() > 0, (method, alpha)
    assert worst <= 1e-10


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_energies_block_256x256x32(env, prec):
    """Per-term FP64 energies at the benchmark's full size (the stray term through the
    512-point y pass and the 64-point convolution)."""
    torch, sg = env
    c = workloads.config("block-256x256x32")
    m = workloads.initial_state(c)
    B = (7e-3, -4e-3, 1e-3)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, prec)
    e = plan.energy(to_dev(torch, m, prec), B)
    P = oracle_problem_si(c.n, c.h, c.dt, ALL)
    eref = scheme.energies(P, rounded_like(m, prec), oracle_field_si(B, ALL))
    mu0ms2 = 4e-7 * np.pi * workloads.MS_PY ** 2
    erel = {k: abs(e[k] / mu0ms2 - eref[k]) / (abs(eref["total"]) + abs(eref[k]) + 1e-30) for k in eref}
    print(f"block energies {'fp64' if prec else 'fp32'}: " + ", ".join(f"{k} {v:.1e}" for k, v in erel.items()))
    for k in eref:
        assert erel[k] <= (1e-11 if prec == 1 else 1e-6), k


def test_projection_flags_non_finite(env):
    torch, sg = env
    n = (8, 4, 1)
    plan = gpu_plan_si(sg, n, CELL, DT, ALL, 0)
    m = workloads.random_unit((1, 4, 8), 105)
    m[:, 0, 2, 3] = np.nan
    md = to_dev(torch, m, 0)
    plan.step(md, 0.01, (0.0, 0.0, 0.0))
    with pytest.raises(sg.SGSPMError) as e:
        plan.check()
    assert e.value.code == -5
    plan.check()  # flag was cleared


def test_bitwise_deterministic(env):
    torch, sg = env
    c = workloads.config("wall-strip-512x32x4")
    m0 = workloads.initial_state(c)
    plan = gpu_plan_si(sg, c.n, c.h, c.dt, ALL, 0)
    a = _run_gpu(plan, torch, m0, 0.01, [(5e-3, 0, 0)] * 5, 0)
    b = _run_gpu(plan, torch, m0, 0.01, [(5e-3, 0, 0)] * 5, 0)
    assert np.array_equal(a, b)
    e1 = plan.energy(to_dev(torch, a, 0), (5e-3, 0, 0))
    e2 = plan.energy(to_dev(torch, a, 0), (5e-3, 0, 0))
    assert e1 == e2
