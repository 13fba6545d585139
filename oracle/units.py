"""SI -> non-dimensional units for the Landau-Lifshitz equation (oracle side).

The paper works in the non-dimensional form of §2 (eq. c1-large): m_t = -m x h -
alpha m x (m x h) with h = eps Lap m - Q (m2 e2 + m3 e3) + h_s + h_e and states no
material constants.  Reading used here (the usual micromagnetic scaling):
  fields in units of Ms          h_e = B / (mu0 Ms)
  exchange  eps = 2 A / (mu0 Ms^2)   [m^2]   (lengths stay in metres)
  anisotropy Q = 2 K / (mu0 Ms^2)          (easy axis e1 = x, §2)
  time      t = gamma mu0 Ms t_phys
Energies returned by the oracle are the non-dimensional energy times the cell
volume in m^3; multiply by mu0 Ms^2 for joules.
"""
import math

MU0 = 4.0e-7 * math.pi
GAMMA = 1.7609e11  # rad / (s T)


def reduce_si(A, Ms, Ku, dt_seconds):
    """Return (eps [m^2], Q, dt_reduced, t0 [s])."""
    scale = MU0 * Ms * Ms
    eps = 2.0 * A / scale
    Q = 2.0 * Ku / scale
    t0 = 1.0 / (GAMMA * MU0 * Ms)
    return eps, Q, dt_seconds / t0, t0


def field_from_tesla(B, Ms):
    """Applied flux density B [T] -> non-dimensional h_e."""
    return B / (MU0 * Ms)
