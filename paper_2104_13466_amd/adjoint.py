"""Differentiable central-difference rollout: J = 1/2 ||u_K - u*||^2 through K
explicit steps as a function of per-element Lame fields, with the hand-written
discrete adjoint of libsdme behind a ``torch.autograd.Function``.

Forward: u_1 = u_0 + dt v_0 + dt^2/2 a_0, u_{n+1} = 2 u_n - u_{n-1} + dt^2 a_n
(central difference, Section 4), every step one ``sdme_explicit_step`` call;
the pair (u_n, u_{n+1}) is kept every ``checkpoint`` steps.  Backward: the
segments are replayed newest first from their checkpoint and the adjoint
recursion runs through ``sdme_explicit_adjoint_step`` (one mass solve, one
tangent action and one element-sensitivity kernel per step).  All arithmetic
runs in libsdme; this module only orders the calls and holds the buffers.
"""
import torch

from .sdme import FP64


class RolloutSpec:
    """Fixed data of a rollout: context, density, initial state, step, target."""

    def __init__(self, ctx, rho, u0, v0, dt, steps, target, checkpoint=10, mass_rtol=1e-13,
                 prec_force=FP64):
        self.ctx, self.rho, self.u0, self.v0 = ctx, rho, u0, v0
        self.dt, self.K, self.target = dt, steps, target
        self.checkpoint, self.mass_rtol, self.prec_force = checkpoint, mass_rtol, prec_force
        self.stats = {"mass_iterations": 0}


def _step(spec, mat, u_prev, u_cur, u_next):
    st = spec.ctx.explicit_step(mat, spec.prec_force, u_prev, u_cur, u_next, spec.dt,
                                v0=spec.v0 if u_prev is None else None, mass_rtol=spec.mass_rtol)
    spec.stats["mass_iterations"] += st["mass_iterations"]


def rollout(spec, mu, lam, keep=True):
    """Run K steps; return (J, u_K, checkpoints {n: (u_n, u_{n+1})})."""
    mat = spec.ctx.material(mu, lam, spec.rho)
    ckpt = {}
    u_prev, u_cur = None, spec.u0.clone()
    u_next = torch.empty_like(u_cur)
    _step(spec, mat, None, u_cur, u_next)  # u_1
    n = 0
    u_prev, u_cur = u_cur, u_next
    if keep:
        ckpt[0] = (u_prev.clone(), u_cur.clone())
    for n in range(1, spec.K):
        u_next = torch.empty_like(u_cur)
        _step(spec, mat, u_prev, u_cur, u_next)
        u_prev, u_cur = u_cur, u_next
        if keep and n % spec.checkpoint == 0 and n < spec.K - 1:
            ckpt[n] = (u_prev.clone(), u_cur.clone())
    lam_K = torch.empty_like(u_cur)
    J = spec.ctx.misfit(u_cur, spec.target, lam_K)
    return J, u_cur, lam_K, ckpt


def _replay(spec, mat, start, stop, pair):
    """States u_start..u_stop from the checkpoint pair (u_start, u_start+1)."""
    states = {start: pair[0], start + 1: pair[1]}
    for n in range(start + 1, stop):
        nxt = torch.empty_like(pair[0])
        _step(spec, mat, states[n - 1], states[n], nxt)
        states[n + 1] = nxt
    return states


def adjoint(spec, mu, lam, lam_K, ckpt):
    """dJ/dmu, dJ/dlam by the reverse recursion
    lam_n = 2 lam_{n+1} - dt^2 K_T(u_n) M^-1 lam_{n+1} - lam_{n+2}."""
    mat = spec.ctx.material(mu, lam, spec.rho)
    g_mu = torch.zeros_like(mu)
    g_lam = torch.zeros_like(lam)
    lam_n1 = lam_K                       # lam_{n+1}
    lam_n2 = torch.zeros_like(lam_K)     # lam_{n+2}
    starts = sorted(ckpt)
    K = spec.K
    for si in range(len(starts) - 1, -1, -1):
        s0 = starts[si]
        s1 = starts[si + 1] if si + 1 < len(starts) else K  # segment covers n in [s0, s1)
        states = _replay(spec, mat, s0, max(s1 - 1, s0 + 1), ckpt[s0])
        for n in range(s1 - 1, s0 - 1, -1):
            first = n == 0
            lam_out = None if first else torch.empty_like(lam_K)
            st = spec.ctx.explicit_adjoint_step(mat, states[n], lam_n1, None if first else lam_n2,
                                                lam_out, spec.dt, first, g_mu, g_lam,
                                                mass_rtol=spec.mass_rtol)
            spec.stats["mass_iterations"] += st["mass_iterations"]
            if not first:
                lam_n2, lam_n1 = lam_n1, lam_out
    return g_mu, g_lam


class SdmeExplicitRollout(torch.autograd.Function):
    """J(mu, lam) with gradients from the libsdme discrete adjoint."""

    @staticmethod
    def forward(fctx, mu, lam, spec):
        J, uK, lam_K, ckpt = rollout(spec, mu, lam, keep=True)
        fctx.spec = spec
        fctx.lam_K = lam_K
        fctx.ckpt = ckpt
        fctx.save_for_backward(mu, lam)
        return torch.tensor(J, dtype=torch.float64, device=mu.device)

    @staticmethod
    def backward(fctx, gJ):
        mu, lam = fctx.saved_tensors
        g_mu, g_lam = adjoint(fctx.spec, mu, lam, fctx.lam_K, fctx.ckpt)
        return gJ * g_mu, gJ * g_lam, None
