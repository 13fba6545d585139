"""Shared test set-up: the same seeded inputs handed to the GPU library and to the oracle.

The GPU side receives SI (or reduced) parameters and converts them itself; the
oracle side converts with its own units module, so the two conversions are
checked against each other too.
"""
import numpy as np

import workloads
from oracle import scheme, units

TERMS = {"exchange": 1, "aniso": 2, "stray": 4, "zeeman": 8}


def term_mask(terms):
    return sum(TERMS[t] for t in terms)


def oracle_problem_si(n, h, dt, terms, A=workloads.A_PY, Ms=workloads.MS_PY, Ku=workloads.K_PY):
    eps, Q, dtr, _ = units.reduce_si(A, Ms, Ku, dt)
    return scheme.Problem(n=tuple(n), h=tuple(h), eps=eps, dt=dtr, Q=Q if "aniso" in terms else 0.0,
                          stray="stray" in terms, exchange="exchange" in terms)


def oracle_field_si(B, terms, Ms=workloads.MS_PY):
    if "zeeman" not in terms:
        return (0.0, 0.0, 0.0)
    return tuple(units.field_from_tesla(b, Ms) for b in B)


def gpu_plan_si(sg, n, h, dt, terms, precision, scheme_=0, A=workloads.A_PY, Ms=workloads.MS_PY,
                Ku=workloads.K_PY):
    return sg.Plan(nx=n[0], ny=n[1], nz=n[2], dx=h[0], dy=h[1], dz=h[2], dt=dt, units=sg.UNITS_SI, A=A,
                   Ms=Ms, Ku=Ku, terms=term_mask(terms), precision=precision, scheme=scheme_)


def gpu_plan_reduced(sg, n, h, dt, eps, Q, terms, precision, scheme_=0):
    return sg.Plan(nx=n[0], ny=n[1], nz=n[2], dx=h[0], dy=h[1], dz=h[2], dt=dt, units=sg.UNITS_REDUCED,
                   eps=eps, Q=Q, terms=term_mask(terms), precision=precision, scheme=scheme_)


def to_dev(torch, a, precision):
    dt = torch.float64 if precision == 1 else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def rounded_like(a, precision):
    """The FP64 values the GPU actually starts from (FP32 plans round their inputs)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64) if precision == 0 else np.asarray(a, np.float64)
