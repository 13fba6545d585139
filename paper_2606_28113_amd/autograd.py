"""Final-state gradients of an SGSPM run behind torch.autograd.Function.

Forward runs S library steps and keeps m every K steps; backward replays each
segment from its checkpoint, keeping every step's tape (sgspm_step_taped), and
pulls the cotangent back one step at a time from those tapes
(sgspm_adjoint_step_taped), so each step runs forward once in the backward
pass.  When the K tapes do not fit in device memory (or TAPED is False) each
adjoint step recomputes its step instead (sgspm_adjoint_step); the gradients
are the same bit for bit.  Gradients: m0 (ambient R^{3N}, no renormalisation),
the applied-field schedule h_e (S, 3) and alpha.
"""
import torch

# keep the tapes of a replayed segment (K tapes of 18 fields each)
TAPED = True


def _tapes(plan, K):
    if not TAPED:
        return None
    try:
        return plan.new_tapes(K)
    except (RuntimeError, torch.cuda.OutOfMemoryError):
        return None


def run_steps(plan, m, alpha, h_e_sched, src=None):
    """Advance m in place by len(h_e_sched) steps."""
    for n in range(len(h_e_sched)):
        plan.step(m, alpha, h_e_sched[n], None if src is None else src[n])
    return m


class SGSPMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, h_e, alpha, plan, ckpt_every):
        he = h_e.detach().to("cpu", torch.float64)
        a = float(alpha)
        S = he.shape[0]
        K = max(1, int(ckpt_every))
        m = m0.detach().clone().contiguous()
        ckpts = {}
        for n in range(S):
            if n % K == 0:
                ckpts[n] = m.clone()
            plan.step(m, a, he[n].tolist(), None)
        ctx.plan, ctx.he, ctx.alpha, ctx.K, ctx.ckpts = plan, he, a, K, ckpts
        ctx.h_e_dtype, ctx.h_e_device = h_e.dtype, h_e.device
        ctx.alpha_is_tensor = torch.is_tensor(alpha)
        if ctx.alpha_is_tensor:
            ctx.alpha_dtype, ctx.alpha_device = alpha.dtype, alpha.device
        return m

    @staticmethod
    def backward(ctx, g):
        plan, he, a, K = ctx.plan, ctx.he, ctx.alpha, ctx.K
        S = he.shape[0]
        lam = g.detach().to(plan.dtype).contiguous().clone()
        gstep = torch.zeros(4, dtype=torch.float64, device=lam.device)
        dhe = torch.zeros((S, 3), dtype=torch.float64, device=lam.device)
        dalpha = torch.zeros((), dtype=torch.float64, device=lam.device)
        tapes = _tapes(plan, K)
        for s0 in sorted(ctx.ckpts.keys(), reverse=True):
            s1 = min(s0 + K, S)
            states = [ctx.ckpts[s0]]
            m = ctx.ckpts[s0].clone()
            if tapes is not None:
                for n in range(s0, s1):
                    plan.step_taped(m, a, he[n].tolist(), tapes[n - s0])
                    if n + 1 < s1:
                        states.append(m.clone())
            else:
                for n in range(s0, s1 - 1):
                    plan.step(m, a, he[n].tolist(), None)
                    states.append(m.clone())
            for n in range(s1 - 1, s0 - 1, -1):
                gstep.zero_()
                if tapes is not None:
                    plan.adjoint_step_taped(states[n - s0], a, he[n].tolist(), tapes[n - s0], lam, gstep)
                else:
                    plan.adjoint_step(states[n - s0], a, he[n].tolist(), lam, gstep)
                dhe[n] = gstep[:3]
                dalpha += gstep[3]
        g_m0 = lam
        g_he = dhe.to(ctx.h_e_dtype).to(ctx.h_e_device)
        g_alpha = dalpha.to(ctx.alpha_dtype).to(ctx.alpha_device) if ctx.alpha_is_tensor else None
        return g_m0, g_he, g_alpha, None, None
