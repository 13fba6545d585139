"""Adjoint and tangent-linear model of one SGSPM step (oracle, FP64).

The paper has no adjoint; this is the chain rule applied to the step of §3.2 as
the oracle computes it (scheme.sgspm_step, including its readings).  Facts used:
  * the solves H = (I - eps dt Lap_h)^{-1} and H_a = (I - alpha eps dt Lap_h)^{-1}
    are symmetric (the mirror-ghost Lap_h is symmetric);
  * the stray operator K u = -N (*) u is symmetric: N_ab = N_ba and every N_ab is
    even under r -> -r, so K^T = K;
  * d H_a / d alpha = H_a (eps dt Lap_h) H_a.
The source term of a manufactured solution is an additive constant and carries
no gradient.  Gradients are in ambient R^{3N} (m0 is not renormalised).
"""
import numpy as np

from . import operators
from .scheme import sgspm_step


def _K(P, v):
    return P.stray_field(np.asarray(v, dtype=np.float64))


def _sum(x):
    return float(np.sum(x))


def adjoint_step(P, m, alpha, h_e, lam, src=None):
    """Pull lam = dL/dm^{n+1} back through one step started at m = m^n.

    Returns (dL/dm^n, dL/dh_e^n (3,), dL/dalpha contribution of this step).
    """
    t = {}
    sgspm_step(P, m, alpha, h_e, src=src, tape=t)
    dt, Q = P.dt, P.Q
    m1, m2, m3 = t["m"]
    g2n, g3n, m1s, g1s = t["g2n"], t["g3n"], t["m1s"], t["g1s"]
    m2s, g2s, m3s = t["m2s"], t["g2s"], t["m3s"]
    g3ss, m2ss, g2ss, m1ss = t["g3ss"], t["m2ss"], t["g2ss"], t["m1ss"]
    u, nrm, c, F = t["m_next"], t["nrm"], t["msss"], t["f_ss"]
    lam = np.asarray(lam, dtype=np.float64)
    dh = np.zeros(3)

    # Step 3 projection c -> c/|c|
    lam_c = (lam - np.sum(lam * u, axis=0) * u) / nrm
    # Step 2 heat flow: c_i = H_a (u_F,i + alpha dt F_i)
    lam_w = np.stack([P.H_alpha(lam_c[i], alpha) for i in range(3)])
    dalpha = dt * _sum(lam_w * (P.eps_eff * operators.laplacian_vec(c, P.h) + F))
    for i in range(3):
        dh[i] += alpha * dt * _sum(lam_w[i])
    lam_F = alpha * dt * lam_w
    lam_uF = lam_w + _K(P, lam_F)
    lam_uF[1] -= Q * lam_F[1]
    lam_uF[2] -= Q * lam_F[2]
    l_m1ss, l_m2ss, l_m3s = lam_uF[0].copy(), lam_uF[1].copy(), lam_uF[2].copy()
    l_m1 = np.zeros_like(m1)
    l_m2 = np.zeros_like(m1)
    l_m3 = np.zeros_like(m1)
    l_m1s = np.zeros_like(m1)
    l_m2s = np.zeros_like(m1)

    # m1** = m1 + g2** m3** - g3** m2**
    l_m1 += l_m1ss
    l_g2ss = l_m1ss * m3s
    l_m3s += l_m1ss * g2ss
    l_g3ss = -l_m1ss * m2ss
    l_m2ss += -l_m1ss * g3ss
    # g2** = H(m2** + dt f2(m1*, m2**, m3**))
    mu = P.H(l_g2ss)
    l_m2ss += (1.0 - dt * Q) * mu
    dh[1] += dt * _sum(mu)
    k = _K(P, np.stack([np.zeros_like(mu), dt * mu, np.zeros_like(mu)]))
    l_m1s += k[0]
    l_m2ss += k[1]
    l_m3s += k[2]
    # m2** = m2 + g3** m1* - g1* m3**
    l_m2 += l_m2ss
    l_g3ss += l_m2ss * m1s
    l_m1s += l_m2ss * g3ss
    l_g1s = -l_m2ss * m3s
    l_m3s += -l_m2ss * g1s
    # g3** = H(m3** + dt f3(m1*, m2*, m3**))
    mu = P.H(l_g3ss)
    l_m3s += (1.0 - dt * Q) * mu
    dh[2] += dt * _sum(mu)
    k = _K(P, np.stack([np.zeros_like(mu), np.zeros_like(mu), dt * mu]))
    l_m1s += k[0]
    l_m2s += k[1]
    l_m3s += k[2]
    # m3* (= m3**) = m3 + g1* m2* - g2* m1*
    l_m3 += l_m3s
    l_g1s += l_m3s * m2s
    l_m2s += l_m3s * g1s
    l_g2s = -l_m3s * m1s
    l_m1s += -l_m3s * g2s
    # g2* = H(m2* + dt f2(m1*, m2*, m3))
    mu = P.H(l_g2s)
    l_m2s += (1.0 - dt * Q) * mu
    dh[1] += dt * _sum(mu)
    k = _K(P, np.stack([np.zeros_like(mu), dt * mu, np.zeros_like(mu)]))
    l_m1s += k[0]
    l_m2s += k[1]
    l_m3 += k[2]
    # m2* = m2 + g3^n m1* - g1* m3
    l_m2 += l_m2s
    l_g3n = l_m2s * m1s
    l_m1s += l_m2s * g3n
    l_g1s += -l_m2s * m3
    l_m3 += -l_m2s * g1s
    # g1* = H(m1* + dt f1(m1*, m2, m3))
    mu = P.H(l_g1s)
    l_m1s += mu
    dh[0] += dt * _sum(mu)
    k = _K(P, np.stack([dt * mu, np.zeros_like(mu), np.zeros_like(mu)]))
    l_m1s += k[0]
    l_m2 += k[1]
    l_m3 += k[2]
    # m1* = m1 + g2^n m3 - g3^n m2
    l_m1 += l_m1s
    l_g2n = l_m1s * m3
    l_m3 += l_m1s * g2n
    l_g3n += -l_m1s * m2
    l_m2 += -l_m1s * g3n
    # g2^n = H(m2 + dt f2(m)), g3^n = H(m3 + dt f3(m))
    mu2 = P.H(l_g2n)
    mu3 = P.H(l_g3n)
    l_m2 += (1.0 - dt * Q) * mu2
    l_m3 += (1.0 - dt * Q) * mu3
    dh[1] += dt * _sum(mu2)
    dh[2] += dt * _sum(mu3)
    k = _K(P, np.stack([np.zeros_like(mu2), dt * mu2, dt * mu3]))
    l_m1 += k[0]
    l_m2 += k[1]
    l_m3 += k[2]
    return np.stack([l_m1, l_m2, l_m3]), dh, dalpha


def tangent_step(P, m, alpha, h_e, dm, dh_e, dalpha, src=None):
    """Directional derivative of sgspm_step at (m, h_e, alpha) along (dm, dh_e, dalpha)."""
    t = {}
    sgspm_step(P, m, alpha, h_e, src=src, tape=t)
    dt, Q = P.dt, P.Q
    m1, m2, m3 = t["m"]
    d1, d2, d3 = (np.asarray(x, dtype=np.float64) for x in dm)
    dh_e = np.asarray(dh_e, dtype=np.float64)

    def df(du, i):
        """Directional derivative of f_i along a state perturbation du."""
        out = _K(P, du)[i] + dh_e[i]
        if i > 0:
            out = out - Q * du[i]
        return out

    g2n, g3n, m1s, g1s = t["g2n"], t["g3n"], t["m1s"], t["g1s"]
    m2s, g2s, m3s, g3ss, m2ss, g2ss = t["m2s"], t["g2s"], t["m3s"], t["g3ss"], t["m2ss"], t["g2ss"]
    dg2n = P.H(d2 + dt * df((d1, d2, d3), 1))
    dg3n = P.H(d3 + dt * df((d1, d2, d3), 2))
    dm1s = d1 + dg2n * m3 + g2n * d3 - dg3n * m2 - g3n * d2
    dg1s = P.H(dm1s + dt * df((dm1s, d2, d3), 0))
    dm2s = d2 + dg3n * m1s + g3n * dm1s - dg1s * m3 - g1s * d3
    dg2s = P.H(dm2s + dt * df((dm1s, dm2s, d3), 1))
    dm3s = d3 + dg1s * m2s + g1s * dm2s - dg2s * m1s - g2s * dm1s
    dg3ss = P.H(dm3s + dt * df((dm1s, dm2s, dm3s), 2))
    dm2ss = d2 + dg3ss * m1s + g3ss * dm1s - dg1s * m3s - g1s * dm3s
    dg2ss = P.H(dm2ss + dt * df((dm1s, dm2ss, dm3s), 1))
    dm1ss = d1 + dg2ss * m3s + g2ss * dm3s - dg3ss * m2ss - g3ss * dm2ss
    duF = np.stack([dm1ss, dm2ss, dm3s])
    F, c, u, nrm = t["f_ss"], t["msss"], t["m_next"], t["nrm"]
    dw = duF + alpha * dt * np.stack([df(duF, i) for i in range(3)]) + dalpha * dt * F
    # c = H_a w  =>  dc = H_a dw + dalpha H_a (eps dt Lap_h c)
    lap_c = operators.laplacian_vec(c, P.h)
    dc = np.stack([P.H_alpha(dw[i] + dalpha * P.eps_eff * dt * lap_c[i], alpha) for i in range(3)])
    return (dc - np.sum(dc * u, axis=0) * u) / nrm


def run_with_grad(P, m0, alpha, h_e_sched, target, src_sched=None):
    """Final-state loss L = mean((m_S - target)^2) and its gradients.

    h_e_sched has shape (S, 3).  Returns (L, dL/dm0, dL/dh_e (S, 3), dL/dalpha).
    Plain reverse sweep over stored states (no checkpointing in the oracle).
    """
    S = len(h_e_sched)
    states = [np.asarray(m0, dtype=np.float64)]
    for n in range(S):
        src = None if src_sched is None else src_sched[n]
        states.append(sgspm_step(P, states[-1], alpha, h_e_sched[n], src=src))
    diff = states[-1] - target
    L = float(np.mean(diff * diff))
    lam = 2.0 * diff / diff.size
    dh = np.zeros((S, 3))
    da = 0.0
    for n in range(S - 1, -1, -1):
        src = None if src_sched is None else src_sched[n]
        lam, dh[n], d = adjoint_step(P, states[n], alpha, h_e_sched[n], lam, src=src)
        da += d
    return L, lam, dh, da
