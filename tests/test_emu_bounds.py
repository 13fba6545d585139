"""Every global and LDS access of the library's kernels, checked on the CPU.

The kernel and plan sources compile with g++ against a host emulation of the
HIP subset they use (tests/emu/): each launch runs its workgroups as fibers,
one per work-item, with __syncthreads and wave shuffles as scheduling points;
device allocations are host allocations of the exact size; the dynamic LDS is
one host array whose bytes beyond the launch's size are poisoned.  Built with
AddressSanitizer, any access outside an allocation or beyond a launch's LDS
aborts the run with the kernel's source line.  The emulator also rejects a
launch with an empty grid, more than 1024 work-items or more than 160 KiB of
LDS, and work-items that wait at different synchronisation points.

Each case creates a plan through the C ABI and calls every entry point once
(steps, energy, unit-length error, step with spectral radii, field, stray field,
demagnetising tensor, heat solve, adjoint step and its allocation-free form).
Small grids run every workgroup, and their FP64 results are compared with the
oracle, which also shows that the emulation keeps the kernels' semantics.
Large grids run a spread sample of workgroups per launch, always including the
first and last along every grid axis, for the bounds check alone.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from helpers import oracle_field_si, oracle_problem_si
from oracle import adjoint as oadj, demag, operators, scheme, spectral, units

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
BUILD = os.path.join(EMU, "_build")
EXE = os.path.join(BUILD, "emu_sgspm")
CSRC = os.path.join(HERE, "..", "paper_2606_28113_amd", "csrc")
INC = os.path.join(HERE, "..", "include")

ALL = 15
CELL = 4e-9
DT = 0.1e-12
ALPHA = 0.02
HE = (5e-3, 1e-3, -2e-3)

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def emu_exe():
    os.makedirs(BUILD, exist_ok=True)
    common = ["g++", "-std=c++17", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address",
              "-I", os.path.join(EMU, "include"), "-I", INC]
    units = [("emu_kernels.cpp", "k.o"), ("emu_plan.cpp", "p.o"), ("emu_runtime.cpp", "r.o"), ("emu_main.cpp", "m.o")]
    deps = [os.path.join(CSRC, f) for f in ("kernels.hip", "kernels.h", "fft_lds.h", "plan.hip")] + \
        [os.path.join(INC, "sgspm.h"), os.path.join(EMU, "include", "hip", "hip_runtime.h")]
    newest_dep = max(os.path.getmtime(d) for d in deps)
    procs = []
    for src, obj in units:
        o = os.path.join(BUILD, obj)
        s = os.path.join(EMU, src)
        if os.path.exists(o) and os.path.getmtime(o) > max(newest_dep, os.path.getmtime(s)):
            continue
        procs.append((src, subprocess.Popen(common + ["-c", s, "-o", o], stderr=subprocess.PIPE, text=True)))
    for src, p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, f"{src}:\n{err[-4000:]}"
    subprocess.run(["g++", "-fsanitize=address"] + [os.path.join(BUILD, o) for _, o in units] + ["-o", EXE],
                   check=True)
    return EXE


def _inputs(shape, seed):
    m0 = workloads.random_unit(shape, seed)
    lam = np.random.default_rng(seed + 1).normal(size=(3,) + shape)
    return m0, lam


def _run(exe, tmp_path, n, prec, scheme_=0, terms=ALL, steps=2, sample=0, seed=300):
    shape = (n[2], n[1], n[0])
    m0, lam = _inputs(shape, seed)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([m0.ravel(), lam.ravel()]).tofile(fin)
    env = dict(os.environ, EMU_MAX_GROUPS=str(sample),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0")
    args = [exe] + [str(v) for v in (n[0], n[1], n[2], prec, scheme_, terms, steps, workloads.A_PY,
                                     workloads.MS_PY, workloads.K_PY, CELL, DT, ALPHA, *HE)] + [str(fin), str(fout)]
    print("emulating", " ".join(args[1:-2]), "sample", sample, flush=True)
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "ERROR" not in r.stderr, r.stderr[-6000:]
    out = np.fromfile(fout)
    N = int(np.prod(shape))
    parts = {}
    k = 0
    for name, size in (("m", 3 * N), ("energy", 5), ("unit_error", 1), ("rho", 2), ("h_eff", 3 * N),
                       ("h_s", 3 * N), ("heat", N), ("lam", 3 * N), ("grad", 4), ("lam_na", 3 * N),
                       ("grad_na", 4)):
        parts[name] = out[k:k + size]
        k += size
    assert k == out.size
    for name in ("m", "h_eff", "h_s", "heat", "lam", "lam_na"):
        parts[name] = parts[name].reshape(((3,) if name != "heat" else ()) + shape)
    return m0, lam, parts


# the grid shapes of the generic kernels (power-of-two and mixed-radix extents,
# films, lines and single cells) and rows of 256 (the 512-point register row
# kernels; an odd number of rows, whose x-major heat arrays the register kernels
# cannot pair, goes to the generic ones), every workgroup, FP64, against the oracle
FULL = [(16, 8, 4), (12, 10, 3), (4, 1, 8), (30, 1, 1), (1, 1, 1), (256, 2, 1), (256, 3, 1)]
# and (SGSPM_EMU_ALL=1) the special extents (rows of 256, the 256-point y pass) mixed
# with odd ones
FULL_MORE = [(8, 4, 2), (1, 16, 1), (6, 5, 1), (256, 5, 3), (256, 1, 3), (256, 3, 5), (3, 256, 1), (5, 256, 3),
             (256, 2, 3)]
# SGSPM_EMU_ALL=1 adds the longer lists below to the default ones
EMU_ALL = os.environ.get("SGSPM_EMU_ALL") == "1"


@pytest.mark.parametrize("n", FULL + (FULL_MORE if EMU_ALL else []), ids=lambda n: "x".join(map(str, n)))
def test_every_access_in_bounds_fp64(emu_exe, tmp_path, n):
    m0, lam, got = _run(emu_exe, tmp_path, n, 1)
    P = oracle_problem_si(n, (CELL,) * 3, DT, ("exchange", "aniso", "stray", "zeeman"))
    he = oracle_field_si(HE, ("zeeman",))
    m = m0
    for _ in range(2):
        m = scheme.sgspm_step(P, m, ALPHA, he)
    assert np.abs(got["m"] - m).max() <= 1e-10
    hs = demag.stray_field(m0, demag.kernel_spectra(m0.shape[1:], (CELL,) * 3))
    assert np.abs(got["h_s"] - hs).max() <= 1e-10
    assert np.abs(got["h_eff"] - scheme.effective_field(P, m0, he)).max() <= 1e-10 * max(1.0, P.eps / min(P.h) ** 2)
    g = operators.heat_solve(m0[0], P.eps * P.dt, P.h)
    assert np.abs(got["heat"] - g).max() <= 1e-12
    rho = spectral.spectral_radii(P, m0, ALPHA, he)
    assert got["rho"] == pytest.approx(rho, rel=1e-9, abs=1e-14)
    lref, dh, da = oadj.adjoint_step(P, m0, ALPHA, he, lam)
    assert np.abs(got["lam"] - lref).max() <= 1e-11 * np.abs(lref).max()
    fscale = 1.0 / (units.MU0 * workloads.MS_PY)   # reduced field per tesla
    assert np.allclose(got["grad"][:3], dh * fscale, rtol=1e-10, atol=1e-12 * np.abs(dh * fscale).max())
    assert got["grad"][3] == pytest.approx(da, rel=1e-10, abs=1e-14)
    # the allocation-free adjoint is the same computation
    assert np.array_equal(got["lam"], got["lam_na"]) and np.array_equal(got["grad"], got["grad_na"])


@pytest.mark.skipif(not EMU_ALL, reason="longer emulation list (SGSPM_EMU_ALL=1)")
@pytest.mark.parametrize("n", [(16, 8, 4), (12, 10, 3), (256, 2, 1)], ids=lambda n: "x".join(map(str, n)))
def test_every_access_in_bounds_fp32(emu_exe, tmp_path, n):
    m0, _, got = _run(emu_exe, tmp_path, n, 0)
    P = oracle_problem_si(n, (CELL,) * 3, DT, ("exchange", "aniso", "stray", "zeeman"))
    he = oracle_field_si(HE, ("zeeman",))
    m = np.asarray(m0, np.float32).astype(np.float64)
    for _ in range(2):
        m = scheme.sgspm_step(P, m, ALPHA, he)
    assert np.abs(got["m"] - m).max() <= 1e-5


@pytest.mark.parametrize("sch", [1, 2], ids=["gspm", "sgspm_ff"])
def test_every_access_in_bounds_other_schemes(emu_exe, tmp_path, sch):
    n = (12, 8, 2)
    m0, _, got = _run(emu_exe, tmp_path, n, 1, scheme_=sch)
    P = oracle_problem_si(n, (CELL,) * 3, DT, ("exchange", "aniso", "stray", "zeeman"))
    he = oracle_field_si(HE, ("zeeman",))
    step = scheme.gspm_step if sch == 1 else scheme.sgspm_ff_step
    m = m0
    for _ in range(2):
        m = step(P, m, ALPHA, he)
    assert np.abs(got["m"] - m).max() <= 1e-10


# workload grids and the register kernels' grids: a spread sample of workgroups
# per launch (first and last along every grid axis included), bounds only
SAMPLED = [((512, 32, 4), 0, ALL), ((100, 100, 4), 1, ALL), ((2000, 1, 1), 1, 1), ((256, 256, 32), 0, ALL)]
if EMU_ALL:
    SAMPLED += [((128, 64, 1), 0, ALL), ((100, 100, 4), 0, ALL), ((2000, 1, 1), 0, 1), ((256, 8, 32), 0, ALL),
                ((16, 256, 32), 1, ALL), ((256, 256, 32), 1, ALL), ((128, 128, 1), 1, ALL)]


@pytest.mark.parametrize("n,prec,terms", SAMPLED,
                         ids=["x".join(map(str, n)) + ("-fp64" if p else "-fp32") + ("" if t == ALL else "-exchange")
                              for n, p, t in SAMPLED])
def test_every_sampled_access_in_bounds(emu_exe, tmp_path, n, prec, terms):
    _run(emu_exe, tmp_path, n, prec, terms=terms, steps=1, sample=6)


# extremes of what sgspm_validate accepts: every accepted parameter set must plan
# and run without a launch-geometry error or an access out of bounds, and every
# rejected one must be rejected before any launch
EXTREMES = [(1024, 2, 1), (2048, 1, 1), (2, 2, 512), (4, 1024, 2), (1000, 3, 1), (5, 3, 640), (1280, 2, 2)]
if EMU_ALL:
    EXTREMES += [(1024, 1, 1), (2, 512, 1), (2, 256, 1), (2, 2, 256), (2, 1024, 1), (1, 1, 1024), (1, 1024, 1),
                 (6, 750, 1), (2000, 1, 1), (512, 512, 1), (16, 16, 256), (3, 5, 15), (1024, 16, 32)]


@pytest.mark.parametrize("terms", [ALL, 1] if EMU_ALL else [ALL], ids=["all", "exchange"][:2 if EMU_ALL else 1])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("n", EXTREMES, ids=lambda n: "x".join(map(str, n)))
def test_validated_extremes_run(emu_exe, tmp_path, n, prec, terms):
    import paper_2606_28113_amd as sg
    try:
        sg.validate(nx=n[0], ny=n[1], nz=n[2], dx=CELL, dy=CELL, dz=CELL, dt=DT, units=sg.UNITS_SI,
                    A=workloads.A_PY, Ms=workloads.MS_PY, Ku=workloads.K_PY, terms=terms, precision=prec)
    except sg.SGSPMError as e:
        assert e.code == -2, str(e)
        return
    _run(emu_exe, tmp_path, n, prec, terms=terms, steps=1, sample=2)


def _run_batch(exe, tmp_path, n, prec, B, scheme_=0, steps=2, seed=310):
    shape = (n[2], n[1], n[0])
    m0, lam = _inputs(shape, seed)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([m0.ravel(), lam.ravel()]).tofile(fin)
    env = dict(os.environ, EMU_MAX_GROUPS="0", EMU_BATCH=str(B),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0")
    args = [exe] + [str(v) for v in (n[0], n[1], n[2], prec, scheme_, ALL, steps, workloads.A_PY,
                                     workloads.MS_PY, workloads.K_PY, CELL, DT, ALPHA, *HE)] + [str(fin), str(fout)]
    print("emulating batch", B, " ".join(args[1:-2]), flush=True)
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    out = np.fromfile(fout)
    N = int(np.prod(shape))
    mb = out[:3 * B * N].reshape((3, B) + shape)
    eb = out[3 * B * N:3 * B * N + 5 * B].reshape(B, 5)
    eb0 = out[3 * B * N + 5 * B:3 * B * N + 10 * B].reshape(B, 5)
    rest = out[3 * B * N + 10 * B:].reshape(B, 5 + 3 * N + 5)
    return mb, eb, eb0, rest[:, 5:5 + 3 * N].reshape((B, 3) + shape), rest[:, 5 + 3 * N:], rest[:, :5]


# batched plans (runs sharing every launch): every run equals its single-run plan
# bit for bit, states and energies; 3-D with the y pass, a film, mixed radix, rows
# of 256 (register row kernels in single precision), several y-z planes per
# workgroup (1024 x 2 x 2), both schemes
BATCH_CASES = [((16, 8, 4), 1, 3, 0, "16x8x4-fp64-B3"), ((1024, 2, 2), 0, 2, 0, "1024x2x2-fp32-B2")]
if EMU_ALL:
    BATCH_CASES += [((12, 10, 2), 0, 2, 0, "12x10x2-fp32-B2"), ((16, 8, 1), 1, 2, 1, "16x8x1-fp64-B2-gspm"),
                    ((256, 2, 2), 0, 2, 0, "256x2x2-fp32-B2")]


@pytest.mark.parametrize("n,prec,B,sch", [c[:4] for c in BATCH_CASES], ids=[c[4] for c in BATCH_CASES])
def test_batched_runs_match_single_runs(emu_exe, tmp_path, n, prec, B, sch):
    mb, eb, eb0, ms, es, es0 = _run_batch(emu_exe, tmp_path, n, prec, B, scheme_=sch)
    for b in range(B):
        assert np.array_equal(mb[:, b], ms[b]), b
        assert np.array_equal(eb[b], es[b]), b
        assert np.array_equal(eb0[b], es0[b]), b
    assert not np.array_equal(ms[0], ms[1])
