"""Seeded synthetic workloads for the SGSPM time step.

Inputs only: grids, material constants, step counts, initial magnetisations and
applied-field schedules.  Nothing here performs any arithmetic of the method
(no solves, no fields, no time steps); both the GPU library's callers and the
CPU oracle's tests draw their inputs from this module.

Five configurations, shaped like the paper's runs (§5: manufactured solution,
thin films, a Neel-wall strip) plus a large block for bandwidth measurements:

  mf-film-32x32           32x32x1 on [0,1]^2, reduced units, exchange only (eps = 0.1), alpha = 0.01,
      dt = 1e-3, 200 steps, manufactured solution with forcing; m0 = exact(t=0)
      + N(0, 1e-3^2) noise, renormalised (seed 1).
  film-128x64             128x64x1 film, 4 nm cells, permalloy-like (A = 1.3e-11 J/m, Ms = 8e5 A/m,
      K = 500 J/m^3 along x), all four fields, 5 mT along +x, alpha = 0.01,
      dt = 0.1 ps, 1000 steps, m0 i.i.d. uniform on the sphere (seed 2).
  wall-strip-512x32x4     512x32x4 strip, same material, tanh Neel wall along x of width 20 nm at
      mid-strip plus 1e-3 transverse noise (seed 3); fields 1..20 mT (5 values)
      along +x, alpha in {1e-2, 1e-3, 1e-4}, dt = 0.1 ps, 5000 steps.
  adjoint-film-128x128    128x128x1 film, all fields, alpha = 0.01, dt = 0.1 ps, 500 steps;
      h_e^n = 5 mT e1 + N(0, (0.5 mT)^2) per step and component (seed 4);
      m0 random unit (seed 40), target random unit (seed 41); checkpoints every 50.
  block-256x256x32        256x256x32 block, 4 nm cells, all fields, alpha = 1e-3, dt = 0.05 ps,
      2000 steps, rotating field 10 mT (cos 2 pi f t, sin 2 pi f t, 0), f = 1 GHz;
      m0 = random unit vectors (seed 5) smoothed by 3 passes of a 3-point box
      filter along each axis and renormalised; adjoint over 200 steps, target
      seed 51, checkpoints every 20.
"""
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

A_PY = 1.3e-11   # J/m
MS_PY = 8.0e5    # A/m
K_PY = 500.0     # J/m^3, easy axis x
CELL = 4e-9      # m


@dataclass
class Config:
    name: str
    n: tuple                 # (nx, ny, nz)
    h: tuple                 # (dx, dy, dz)  metres (SI) or reduced lengths
    units: str               # "si" or "reduced"
    dt: float                # seconds (SI) or reduced
    steps: int
    alpha: float
    terms: tuple = ("exchange", "aniso", "stray", "zeeman")
    A: float = A_PY
    Ms: float = MS_PY
    Ku: float = K_PY
    eps: float = 0.0         # reduced units only
    Q: float = 0.0           # reduced units only
    ckpt_every: Optional[int] = None
    adjoint_steps: Optional[int] = None
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    @property
    def cells(self):
        return self.n[0] * self.n[1] * self.n[2]


def config(name):
    if name == "mf-film-32x32":
        return Config("mf-film-32x32", (32, 32, 1), (1 / 32, 1 / 32, 1.0), "reduced", 1e-3, 200, 0.01,
                      terms=("exchange",), eps=0.1, Q=0.0)
    if name == "film-128x64":
        return Config("film-128x64", (128, 64, 1), (CELL,) * 3, "si", 0.1e-12, 1000, 0.01)
    if name == "wall-strip-512x32x4":
        return Config("wall-strip-512x32x4", (512, 32, 4), (CELL,) * 3, "si", 0.1e-12, 5000, 0.01,
                      extra={"fields_mT": list(np.linspace(1.0, 20.0, 5)),
                             "alphas": [1e-2, 1e-3, 1e-4]})
    if name == "adjoint-film-128x128":
        return Config("adjoint-film-128x128", (128, 128, 1), (CELL,) * 3, "si", 0.1e-12, 500, 0.01, ckpt_every=50,
                      adjoint_steps=500)
    if name == "block-256x256x32":
        return Config("block-256x256x32", (256, 256, 32), (CELL,) * 3, "si", 0.05e-12, 2000, 1e-3, ckpt_every=20,
                      adjoint_steps=200)
    raise KeyError(name)


CONFIGS = ("mf-film-32x32", "film-128x64", "wall-strip-512x32x4", "adjoint-film-128x128", "block-256x256x32")


def random_unit(shape, seed):
    """I.i.d. uniform unit vectors: normalised standard normals, shape (3, *shape)."""
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(3,) + tuple(shape))
    return m / np.sqrt(np.sum(m * m, axis=0))


def normalise(v):
    return v / np.sqrt(np.sum(v * v, axis=0))


def box_smoothed_unit(shape, seed, passes=3):
    """Random unit vectors smoothed by a 3-point box filter (edge-replicated) per axis."""
    m = random_unit(shape, seed)
    for _ in range(passes):
        for ax in (1, 2, 3):
            if m.shape[ax] == 1:
                continue
            lo = np.take(m, [0], axis=ax)
            hi = np.take(m, [m.shape[ax] - 1], axis=ax)
            ext = np.concatenate([lo, m, hi], axis=ax)
            n = m.shape[ax]
            m = (np.take(ext, range(0, n), axis=ax) + np.take(ext, range(1, n + 1), axis=ax)
                 + np.take(ext, range(2, n + 2), axis=ax)) / 3.0
    return normalise(m)


def neel_wall(shape, dx, width=20e-9, noise=1e-3, seed=3):
    """(-tanh xi, sech xi, 0) + N(0, noise^2) transverse noise, xi = (x - L/2)/width."""
    nz, ny, nx = shape
    x = (np.arange(nx) + 0.5) * dx
    xi = (x - 0.5 * nx * dx) / width
    m = np.zeros((3,) + tuple(shape))
    m[0] = -np.tanh(xi)[None, None, :]
    m[1] = (1.0 / np.cosh(xi))[None, None, :]
    rng = np.random.default_rng(seed)
    m[1:] += noise * rng.normal(size=(2,) + tuple(shape))
    return normalise(m)


def paper_ic(shape):
    """The paper's exchange-test state, eq. (m0-1): (cos(cos pi x) sin 0.01, sin(cos pi x) sin 0.01, cos 0.01),
    x = (i + 1/2) / nx along the grid's x axis."""
    nz, ny, nx = shape
    x = (np.arange(nx) + 0.5) / nx
    c = np.broadcast_to(np.cos(np.pi * x), tuple(shape))
    return np.stack([np.cos(c) * np.sin(0.01), np.sin(c) * np.sin(0.01), np.full(tuple(shape), np.cos(0.01))])


def c1_initial(shape, seed=1, noise=1e-3):
    """Exact manufactured solution at t = 0 (the constant e3) plus N(0, noise^2), renormalised."""
    rng = np.random.default_rng(seed)
    m = np.zeros((3,) + tuple(shape))
    m[2] = 1.0
    return normalise(m + noise * rng.normal(size=m.shape))


def c4_field_schedule(steps, seed=4):
    """Tesla, shape (steps, 3): 5 mT e1 plus N(0, (0.5 mT)^2) per step and component."""
    rng = np.random.default_rng(seed)
    B = 0.5e-3 * rng.normal(size=(steps, 3))
    B[:, 0] += 5e-3
    return B


def c5_field_schedule(steps, dt, amp=10e-3, freq=1e9):
    """Tesla, shape (steps, 3): rotating in-plane field at step times t_n = n dt."""
    t = np.arange(steps) * dt
    w = 2 * math.pi * freq * t
    return np.stack([amp * np.cos(w), amp * np.sin(w), np.zeros(steps)], axis=1)


def initial_state(cfg, seed=None):
    c = cfg.name
    if c == "mf-film-32x32":
        return c1_initial(cfg.shape)
    if c == "film-128x64":
        return random_unit(cfg.shape, 2 if seed is None else seed)
    if c == "wall-strip-512x32x4":
        return neel_wall(cfg.shape, cfg.h[0])
    if c == "adjoint-film-128x128":
        return random_unit(cfg.shape, 40 if seed is None else seed)
    if c == "block-256x256x32":
        return box_smoothed_unit(cfg.shape, 5 if seed is None else seed)
    raise KeyError(c)


def target_state(cfg):
    return random_unit(cfg.shape, {"adjoint-film-128x128": 41, "block-256x256x32": 51}[cfg.name])


def field_schedule(cfg, steps=None):
    """Applied flux density per step in tesla (SI configs) or reduced h_e (the manufactured film)."""
    steps = cfg.steps if steps is None else steps
    if cfg.name == "mf-film-32x32":
        return np.zeros((steps, 3))
    if cfg.name == "adjoint-film-128x128":
        return c4_field_schedule(steps)
    if cfg.name == "block-256x256x32":
        return c5_field_schedule(steps, cfg.dt)
    B = np.zeros((steps, 3))
    B[:, 0] = 5e-3
    return B
