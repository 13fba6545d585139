"""Plain FP64 CPU oracle for the symmetric Gauss-Seidel projection method (SGSPM).

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library, never to
stand in for it: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP path (``paper_2606_28113_amd``) and imports nothing from it.

Every function is written from the paper (Miao & Xie, "Improved Energy Stable
Symmetric Gauss-Seidel Projection Method for Micromagnetics Simulations"),
citing the section / equation it follows, in FP64, with NumPy/SciPy primitives
(DCT, FFT) as single steps and no blocking or fusion beyond the paper's own
algebra.  Where the paper is silent the module docstrings name the reading
taken.

Array layout everywhere: scalar fields ``(nz, ny, nx)`` with x fastest; vector
fields ``(3, nz, ny, nx)``; the component order is (m1, m2, m3) = (x, y, z).

Modules
  units         SI -> the paper's non-dimensional form
  operators     Neumann Laplacian and the heat-type solve (I - c Lap_h)^-1
  demag         Newell cell-averaged demagnetising tensor and the stray field
  scheme        one SGSPM step (latest-state and frozen-field readings), one GSPM step, energies
  spectral      spectral radius of the Gauss-Seidel / symmetric Gauss-Seidel sweep matrices
  adjoint       reverse (adjoint) and tangent-linear SGSPM step
  manufactured  exact solutions with forcing from the accuracy section

Pinned functions: all (see tests/test_oracle_*.py).  The stray field update
points inside the sweeps (the "latest state" reading, and the frozen-field
reading) are pinned only by self-consistency and by first-order convergence to
the semi-discrete equation: the paper prints no number with the stray field
on, so those readings are "parity unpinned" beyond the invariants the tests
check.  The paper's printed spectral radii are not reproduced (see spectral);
the sweep matrices are pinned by reproducing the step itself.
"""
from . import units, operators, demag, scheme, adjoint, manufactured, spectral  # noqa: F401
from .scheme import Problem, sgspm_step, sgspm_ff_step, gspm_step, energies, effective_field  # noqa: F401
