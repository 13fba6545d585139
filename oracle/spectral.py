"""Spectral radius of the Gauss-Seidel and symmetric Gauss-Seidel sweep matrices (oracle).

Paper §4 writes Step 1 in matrix form for exchange only (eps = 1, f = 0): with
the coefficients c_i^s = dt Lap_h g_i^s, the forward sweep solves
(D - L) m* = U m^n + m^n (eq. GS-matrix) and the backward sweep
(D - U) m** = L m* + m^n (eq. SGS-matrix); the iteration matrices are
G_GS = (D - L)^{-1} U and G_SGS = (D - U)^{-1} L (D - L)^{-1} U, and the paper
reports their spectral radius rho = max |lambda| per step.  Every entry acts
cell by cell, so each cell carries its own 3x3 matrices and rho over the grid is
the largest cell value.

Readings:
  * For a general eps the coefficient is the exchange part of the sweep
    increment, c_i^s = eps dt Lap_h g_i^s (with f on it is the same definition:
    the field part of the increment does not multiply a component).
  * D - U: the paper prints its off-diagonal entries with the signs of D + U.
    The splitting A = D - L - U of the matrix of eq. M (whose strictly upper
    part is [[0, c3, -c2], [0, 0, c1], [0, 0, 0]]) and the scalar backward
    equations of §4 both give D - U = [[1, c3**, -c2**], [0, 1, c1*], [0, 0, 1]];
    that is the form used (the printed L agrees with both).
  * The printed tables of rho (GS-SGS-rad-1D / -3D) are not reproduced by these
    definitions on the grids the accuracy tables use (the 2x2x2 manufactured run
    has a uniform field, where every coefficient vanishes); the values are
    therefore not used as pins (parity of the printed numbers unpinned).
"""
import numpy as np

from . import operators
from .scheme import sgspm_step


def coefficients(P, tape):
    """c_i^s = eps dt Lap_h g_i^s for the six solves of an SGSPM step's tape."""
    k = P.eps_eff * P.dt
    return {s: k * operators.laplacian(tape[s], P.h) for s in ("g2n", "g3n", "g1s", "g2s", "g3ss", "g2ss")}


def sweep_matrices(c):
    """Per-cell (D - L, U, D - U, L), each an array (cells, 3, 3)."""
    c2n, c3n, c1s, c2s, c3ss, c2ss = (np.ravel(c[s]) for s in ("g2n", "g3n", "g1s", "g2s", "g3ss", "g2ss"))
    n = c2n.size
    DL = np.zeros((n, 3, 3))
    U = np.zeros((n, 3, 3))
    DU = np.zeros((n, 3, 3))
    L = np.zeros((n, 3, 3))
    for i in range(3):
        DL[:, i, i] = 1.0
        DU[:, i, i] = 1.0
    # forward sweep, eq. GS-matrix
    DL[:, 1, 0] = -c3n
    DL[:, 2, 0] = c2s
    DL[:, 2, 1] = -c1s
    U[:, 0, 1] = -c3n
    U[:, 0, 2] = c2n
    U[:, 1, 2] = -c1s
    # backward sweep, eq. SGS-matrix (D - U with the splitting's signs, see above)
    DU[:, 0, 1] = c3ss
    DU[:, 0, 2] = -c2ss
    DU[:, 1, 2] = c1s
    L[:, 1, 0] = c3ss
    L[:, 2, 0] = -c2s
    L[:, 2, 1] = c1s
    return DL, U, DU, L


def iteration_matrices(c):
    DL, U, DU, L = sweep_matrices(c)
    G_gs = np.linalg.solve(DL, U)
    G_sgs = np.linalg.solve(DU, L @ G_gs)
    return G_gs, G_sgs


def spectral_radii(P, m, alpha, h_e, src=None):
    """(rho(G_GS), rho(G_SGS)) of the step from m: the largest |eigenvalue| over cells."""
    tape = {}
    sgspm_step(P, m, alpha, h_e, src=src, tape=tape)
    G_gs, G_sgs = iteration_matrices(coefficients(P, tape))
    return (float(np.abs(np.linalg.eigvals(G_gs)).max()), float(np.abs(np.linalg.eigvals(G_sgs)).max()))
