"""CPU-only checks of the C ABI: the library loads, exports every declared entry
point, validates parameters on the host and reduces SI units like the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgspm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(sgspm_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    from paper_2606_28113_amd import binding
    assert _declared() == sorted(binding.EXPORTS)


def test_kernel_classes_match_header():
    """The binding's timing-class names follow the header's SGSPM_KC_* order."""
    from paper_2606_28113_amd import binding
    text = open(HEADER).read()
    kc = dict((n, int(v)) for n, v in re.findall(r"SGSPM_KC_(\w+)\s*=\s*(\d+)", text))
    count = kc.pop("COUNT")
    assert count == len(binding.KERNEL_CLASSES)
    assert [n.lower() for n, _ in sorted(kc.items(), key=lambda t: t[1])] == list(binding.KERNEL_CLASSES)


def test_library_exports_every_declared_symbol():
    from paper_2606_28113_amd import binding
    lib = ctypes.CDLL(binding.lib_path)
    for name in _declared():
        assert hasattr(lib, name), name


GOOD = dict(nx=128, ny=64, nz=1, dx=4e-9, dy=4e-9, dz=4e-9, dt=1e-13, A=1.3e-11, Ms=8e5, Ku=500.0)


def test_validate_accepts_configs():
    import paper_2606_28113_amd as sg
    import workloads
    for name in workloads.CONFIGS:
        c = workloads.config(name)
        kw = dict(nx=c.n[0], ny=c.n[1], nz=c.n[2], dx=c.h[0], dy=c.h[1], dz=c.h[2], dt=c.dt)
        if c.units == "si":
            kw.update(A=c.A, Ms=c.Ms, Ku=c.Ku)
        else:
            kw.update(units=sg.UNITS_REDUCED, eps=c.eps, Q=c.Q)
        sg.validate(**kw)


@pytest.mark.parametrize("bad,code", [
    (dict(nx=0), -1), (dict(ny=-4), -1), (dict(nx=7), -2), (dict(ny=42), -2), (dict(nz=2048), -2),
    (dict(nx=4096), -2), (dict(nx=1536, precision=1), -2), (dict(nx=2000, ny=1, nz=1, precision=1), -2),
    # FP32 rows of 2000 fit, but the demagnetising tensor is transformed in FP64
    (dict(nx=2000, ny=1, nz=1), -2), (dict(nx=1280, ny=2, nz=2), -2),
    (dict(dx=0.0), -1), (dict(dt=-1.0), -1), (dict(dt=float("nan")), -1), (dict(Ms=0.0), -1),
    (dict(A=-1.0), -1), (dict(units=7), -1), (dict(terms=16), -1), (dict(precision=3), -1),
    (dict(scheme=3), -1), (dict(batch=-1), -1), (dict(batch=257), -1),
    # batched plans: SGS or GS, row pairs of one run, fused y-z planes
    (dict(batch=2, scheme=2), -2), (dict(batch=2, ny=3, nz=1), -2), (dict(batch=2, ny=1024, nz=64), -2),
])
def test_validate_rejects(bad, code):
    import paper_2606_28113_amd as sg
    kw = dict(GOOD)
    kw.update(bad)
    with pytest.raises(sg.SGSPMError) as e:
        sg.validate(**kw)
    assert e.value.code == code


@pytest.mark.parametrize("ok", [
    dict(nx=100, ny=100, nz=4), dict(nx=480, ny=30, nz=5), dict(nx=2000, ny=1, nz=1, terms=1, precision=1),
    dict(nx=2000, ny=1, nz=1, terms=1), dict(nx=3, ny=5, nz=15), dict(nx=1024, ny=256, nz=32),
    dict(nx=1024, ny=1, nz=1, precision=1),
], ids=lambda d: "x".join(str(d[k]) for k in ("nx", "ny", "nz")) + ("-fp64" if d.get("precision") else ""))
def test_validate_accepts_products_of_2_3_5(ok):
    """Grid extents that are products of 2, 3 and 5 (the paper's 100 x 100 x 4 film and its
    2000-cell line among them) pass validation while their rows fit a tile."""
    import paper_2606_28113_amd as sg
    kw = dict(GOOD)
    kw.update(ok)
    sg.validate(**kw)


def test_reduced_constants_match_oracle_units():
    import paper_2606_28113_amd as sg
    from oracle import units
    eps, Q, dt, field, energy = sg.reduced_constants(**GOOD)
    e2, q2, d2, _ = units.reduce_si(1.3e-11, 8e5, 500.0, 1e-13)
    assert eps == pytest.approx(e2, rel=1e-14)
    assert Q == pytest.approx(q2, rel=1e-14)
    assert dt == pytest.approx(d2, rel=1e-14)
    assert field == pytest.approx(units.field_from_tesla(1.0, 8e5), rel=1e-14)
    assert energy == pytest.approx(units.MU0 * 8e5 ** 2, rel=1e-14)
    # published permalloy-like numbers: eps / h^2 = 2.0205, 5 mT -> 4.974e-3, 0.1 ps -> 0.017702
    assert eps / (4e-9) ** 2 == pytest.approx(2.0205, abs=1e-4)
    assert 5e-3 * field == pytest.approx(4.974e-3, abs=1e-6)
    assert dt == pytest.approx(0.017702, abs=1e-6)


def test_terms_switch_constants_off():
    import paper_2606_28113_amd as sg
    kw = dict(GOOD, terms=sg.TERM_STRAY | sg.TERM_ZEEMAN)
    eps, Q, *_ = sg.reduced_constants(**kw)
    assert eps == 0.0 and Q == 0.0


def test_entry_points_reject_a_null_plan():
    """Every entry point that takes a plan returns SGSPM_EINVAL for a NULL plan, before any
    device work (so this runs without a GPU), and leaves a message."""
    from paper_2606_28113_amd import binding
    lib = binding.lib
    d3 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    buf = ctypes.c_void_p(1)   # never dereferenced: the plan check comes first
    nb = ctypes.c_size_t()
    calls = {
        "sgspm_step": lambda: lib.sgspm_step(None, buf, 0.01, d3, None),
        "sgspm_step_taped": lambda: lib.sgspm_step_taped(None, buf, 0.01, d3, buf),
        "sgspm_adjoint_step": lambda: lib.sgspm_adjoint_step(None, buf, 0.01, d3, buf, buf),
        "sgspm_adjoint_step_taped": lambda: lib.sgspm_adjoint_step_taped(None, buf, 0.01, d3, buf, buf, buf),
        "sgspm_adjoint_step_noalloc": lambda: lib.sgspm_adjoint_step_noalloc(None, buf, 0.01, d3, buf, buf),
        "sgspm_tape_bytes": lambda: lib.sgspm_tape_bytes(None, ctypes.byref(nb)),
        "sgspm_heat_solve": lambda: lib.sgspm_heat_solve(None, buf, 1.0, buf),
        "sgspm_stray": lambda: lib.sgspm_stray(None, buf, buf),
    }
    for name, call in calls.items():
        assert call() == binding.EINVAL, name
        assert lib.sgspm_last_error(), name
