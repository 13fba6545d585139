"""One time step of SGSPM (and of GSPM), effective field and energies (oracle, FP64).

Paper §3.2 ("Proposed methods") defines SGSPM as
  Step 1  implicit symmetric Gauss-Seidel: a forward sweep m1* -> m2* -> m3* built
          from g_i^n and g_i^*, then a backward sweep m3** -> m2** -> m1** built
          from g_1^*, g_2^*, g_3^**, g_2^**, every backward update rebased on m^n;
  Step 2  heat flow without constraint: (I - alpha eps dt Lap_h) m*** = m** + alpha dt f**;
  Step 3  projection m^{n+1} = m*** / |m***|,
with g_i^s = (I - eps dt Lap_h)^{-1}(m_i^s + dt f_i^s).  §3.1 gives GSPM (forward
sweep only, then Steps 2 and 3 on m*).  f collects every field except exchange:
f = -Q (m2 e2 + m3 e3) + h_s + h_e (§2 effective field, eqs. heat_flow_f).

Readings where the paper is silent or garbled:
  * "latest state": each f_i^s is evaluated at the most recent value of every
    component when g_i^s is formed (the paper computes h_s from the intermediate
    values, §3.1 remark after eq. projection).  Parity unpinned beyond invariants:
    every printed number in the paper is exchange-only.
  * g_i^** (never written out) is formed like g_i^*.
  * m3** repeats the formula of m3*, so m3** = m3*.
  * the backward sweep is rebased on m^n as printed (also the matrix form, eq. SGS-matrix).
  * h_e is held at its step-n value through the whole step.
  * the optional source s (the forcing f_e of a manufactured solution, §5.1) is
    evaluated at t_n and added as + dt s_i to every component update of Step 1,
    in the forward and in the backward sweep; Step 2 carries no source.  This
    reading reproduces the paper's printed 3-D errors (tables temp_acc_3d and
    cpu) to 9-12 significant digits for both SGSPM and GSPM.
  * |m***| = 0 or non-finite raises FloatingPointError.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import demag, operators


@dataclass
class Problem:
    """Grid, cell size and non-dimensional constants of one simulation.

    n = (nx, ny, nz) cells; h = (dx, dy, dz); eps, Q, dt as in §2/§3;
    stray switches h_s on; exchange False sets eps = 0 (H becomes the identity).
    """
    n: tuple
    h: tuple
    eps: float
    dt: float
    Q: float = 0.0
    stray: bool = False
    exchange: bool = True
    _spec: Optional[tuple] = field(default=None, repr=False)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    @property
    def volume(self):
        return self.h[0] * self.h[1] * self.h[2]

    @property
    def eps_eff(self):
        return self.eps if self.exchange else 0.0

    def spectra(self):
        if self._spec is None:
            self._spec = demag.kernel_spectra(self.shape, self.h)
        return self._spec

    def stray_field(self, m):
        if not self.stray:
            return np.zeros_like(m)
        return demag.stray_field(m, self.spectra())

    def f(self, u, h_e):
        """f(u) = -Q (u2 e2 + u3 e3) + h_s(u) + h_e for a state u = (u1, u2, u3)."""
        u = np.asarray(u, dtype=np.float64)
        out = self.stray_field(u)
        out[1] -= self.Q * u[1]
        out[2] -= self.Q * u[2]
        for i in range(3):
            out[i] += h_e[i]
        return out

    def H(self, r):
        """g = (I - eps dt Lap_h)^{-1} r (precession solve of Step 1)."""
        return operators.heat_solve(r, self.eps_eff * self.dt, self.h)

    def H_alpha(self, r, alpha):
        """(I - alpha eps dt Lap_h)^{-1} r (heat-flow solve of Step 2)."""
        return operators.heat_solve(r, alpha * self.eps_eff * self.dt, self.h)


def effective_field(P, m, h_e):
    """h_eff = eps Lap_h m - Q (m2 e2 + m3 e3) + h_s + h_e (§2)."""
    return P.eps_eff * operators.laplacian_vec(m, P.h) + P.f(m, h_e)


def project(c):
    """Step 3: c / |c| cellwise; zero or non-finite norm raises."""
    nrm = np.sqrt(c[0] ** 2 + c[1] ** 2 + c[2] ** 2)
    if not np.all(np.isfinite(nrm)) or np.any(nrm == 0.0):
        raise FloatingPointError("projection: |m***| is zero or non-finite")
    return c / nrm, nrm


def _source_terms(src, dt, shape):
    """dt * s_i per component (zeros when there is no source)."""
    if src is None:
        return np.zeros((3,) + tuple(shape))
    return dt * np.asarray(src, dtype=np.float64)


def sgspm_step(P, m, alpha, h_e, src=None, tape=None):
    """m^{n+1} from m^n by one SGSPM step (§3.2).  ``tape`` (a dict) receives the stages."""
    m = np.asarray(m, dtype=np.float64)
    dt = P.dt
    m1, m2, m3 = m
    s = _source_terms(src, dt, m.shape[1:])
    # Step 1, forward Gauss-Seidel sweep
    f_n = P.f((m1, m2, m3), h_e)
    g2n = P.H(m2 + dt * f_n[1])
    g3n = P.H(m3 + dt * f_n[2])
    m1s = m1 + (g2n * m3 - g3n * m2) + s[0]
    g1s = P.H(m1s + dt * P.f((m1s, m2, m3), h_e)[0])
    m2s = m2 + (g3n * m1s - g1s * m3) + s[1]
    g2s = P.H(m2s + dt * P.f((m1s, m2s, m3), h_e)[1])
    m3s = m3 + (g1s * m2s - g2s * m1s) + s[2]
    # Step 1, backward Gauss-Seidel sweep (3 -> 2 -> 1, rebased on m^n)
    m3ss = m3 + (g1s * m2s - g2s * m1s) + s[2]
    g3ss = P.H(m3ss + dt * P.f((m1s, m2s, m3ss), h_e)[2])
    m2ss = m2 + (g3ss * m1s - g1s * m3ss) + s[1]
    g2ss = P.H(m2ss + dt * P.f((m1s, m2ss, m3ss), h_e)[1])
    m1ss = m1 + (g2ss * m3ss - g3ss * m2ss) + s[0]
    mss = np.stack([m1ss, m2ss, m3ss])
    # Step 2, heat flow without constraint
    f_ss = P.f(mss, h_e)
    rhs = mss + alpha * dt * f_ss
    msss = np.stack([P.H_alpha(rhs[i], alpha) for i in range(3)])
    # Step 3, projection onto S^2
    m_next, nrm = project(msss)
    if tape is not None:
        tape.update(m=m, g2n=g2n, g3n=g3n, m1s=m1s, g1s=g1s, m2s=m2s, g2s=g2s, m3s=m3s,
                    g3ss=g3ss, m2ss=m2ss, g2ss=g2ss, m1ss=m1ss, f_ss=f_ss, rhs=rhs,
                    msss=msss, nrm=nrm, m_next=m_next)
    return m_next


def sgspm_ff_step(P, m, alpha, h_e, src=None):
    """m^{n+1} from m^n by one SGSPM step under the frozen-field reading of Step 1.

    The sweeps of §3.2 as in sgspm_step, but every f^s of Step 1 (both sweeps)
    is the field of the state at the start of the step, f(m^n), evaluated once;
    Step 2 evaluates f once more, at m**.  This is the other reading of where the
    stray field is computed (the remark after eq. projection in §3.1 ties h_s to
    the intermediate values rather than to each partial update), and the
    efficiency direction the Conclusion points to (the improved GSPM variants
    that cut field evaluations): two stray-field evaluations per step instead of
    six.  The source term is placed as in sgspm_step.
    """
    m = np.asarray(m, dtype=np.float64)
    dt = P.dt
    m1, m2, m3 = m
    s = _source_terms(src, dt, m.shape[1:])
    f_n = P.f((m1, m2, m3), h_e)
    # Step 1, forward sweep with f frozen at m^n
    g2n = P.H(m2 + dt * f_n[1])
    g3n = P.H(m3 + dt * f_n[2])
    m1s = m1 + (g2n * m3 - g3n * m2) + s[0]
    g1s = P.H(m1s + dt * f_n[0])
    m2s = m2 + (g3n * m1s - g1s * m3) + s[1]
    g2s = P.H(m2s + dt * f_n[1])
    m3s = m3 + (g1s * m2s - g2s * m1s) + s[2]
    # Step 1, backward sweep (m3** = m3*, rebased on m^n), same frozen f
    g3ss = P.H(m3s + dt * f_n[2])
    m2ss = m2 + (g3ss * m1s - g1s * m3s) + s[1]
    g2ss = P.H(m2ss + dt * f_n[1])
    m1ss = m1 + (g2ss * m3s - g3ss * m2ss) + s[0]
    mss = np.stack([m1ss, m2ss, m3s])
    # Steps 2 and 3 as in sgspm_step
    rhs = mss + alpha * dt * P.f(mss, h_e)
    msss = np.stack([P.H_alpha(rhs[i], alpha) for i in range(3)])
    return project(msss)[0]


def gspm_step(P, m, alpha, h_e, src=None):
    """m^{n+1} from m^n by one GSPM step (§3.1): forward sweep, heat flow, projection."""
    m = np.asarray(m, dtype=np.float64)
    dt = P.dt
    m1, m2, m3 = m
    s = _source_terms(src, dt, m.shape[1:])
    f_n = P.f((m1, m2, m3), h_e)
    g2n = P.H(m2 + dt * f_n[1])
    g3n = P.H(m3 + dt * f_n[2])
    m1s = m1 + (g2n * m3 - g3n * m2) + s[0]
    g1s = P.H(m1s + dt * P.f((m1s, m2, m3), h_e)[0])
    m2s = m2 + (g3n * m1s - g1s * m3) + s[1]
    g2s = P.H(m2s + dt * P.f((m1s, m2s, m3), h_e)[1])
    m3s = m3 + (g1s * m2s - g2s * m1s) + s[2]
    ms = np.stack([m1s, m2s, m3s])
    rhs = ms + alpha * dt * P.f(ms, h_e)
    mss = np.stack([P.H_alpha(rhs[i], alpha) for i in range(3)])
    return project(mss)[0]


def energies(P, m, h_e):
    """Discrete energy per term (non-dimensional energy x volume).

    The paper's E[m] (§2) is printed without the 1/2 factors that make
    h_eff = -dE/dm hold; the consistent form is used:
      E = eps/2 |grad m|^2 + Q/2 (m2^2 + m3^2) - 1/2 h_s.m - h_e.m, integrated.
    Exchange uses forward differences over interior faces (equal to
    -eps/2 sum m.Lap_h m for the mirror-ghost Laplacian).
    """
    m = np.asarray(m, dtype=np.float64)
    V = P.volume
    ex = 0.0
    if P.eps_eff != 0.0:
        for ax, hi in operators.AXES:
            if m.shape[1 + ax] > 1:
                d = np.diff(m, axis=1 + ax)
                ex += float(np.sum(d * d)) / (P.h[hi] ** 2)
        ex *= 0.5 * P.eps_eff * V
    an = 0.5 * P.Q * V * float(np.sum(m[1] ** 2 + m[2] ** 2))
    st = 0.0
    if P.stray:
        hs = P.stray_field(m)
        st = -0.5 * V * float(np.sum(m * hs))
    ze = -V * float(sum(h_e[i] * np.sum(m[i]) for i in range(3)))
    return {"total": ex + an + st + ze, "exchange": ex, "anisotropy": an,
            "stray": st, "zeeman": ze}
