"""Differentiable rollout of the PFC scheme: torch.autograd.Function whose
backward runs the hand-written adjoint step (``pfc_adjoint_step``).

Forward: ``steps`` time steps of scheme (1.10) from ``phi0`` (bootstrap
phi^{-1} = phi^0), in segments of ``ckpt_every`` steps, keeping the state
(phi^{k-1}, phi^k, mu, omega) at the start of each segment.  Backward:
segments are processed last to first; each is recomputed from its checkpoint
and then walked backwards with one adjoint step per time step, accumulating
d/dphi0 and d/deps.

Both passes run a segment through ``run_segment``, which first clears the
handle's cached coarsest Newton inverse (``pfc_reset_coarse_cache``).  The
cache otherwise carries over from whatever ran before (the rest of the
forward pass, or the later segments' recompute and adjoint steps), and the
chord iteration's last bits with it; with the reset, the recompute repeats
the forward segment's kernels on the same inputs and reproduces its
trajectory bit for bit.
"""
from __future__ import annotations

import torch

from .solver import Solver


def run_segment(solver: Solver, state, count: int):
    """``count`` steps from ``state`` = (phi^{k-1}, phi^k, mu, omega) (not
    modified), starting from a rebuilt coarsest inverse.  Returns
    (phis, mu, omega) with phis = [phi^{k-1}, phi^k, ..., phi^{k+count}]."""
    solver.reset_coarse_cache()
    prev, cur, mu, om = (t.clone() for t in state)
    phis = [prev, cur]
    for _ in range(count):
        nxt, _ = solver.step(phis[-2], phis[-1], mu, om)
        phis.append(nxt)
    return phis, mu, om


class PFCRollout(torch.autograd.Function):
    """phi_T = rollout(phi0, eps); gradients with respect to phi0 and eps.

    ``eps`` is a 0-dim float64 tensor; ``params`` a dict with n, L, dt and
    optional tol, nu1, nu2, cycle, max_cycles, adj_tol."""

    @staticmethod
    def forward(ctx, phi0, eps, params, steps, ckpt_every=5):
        p = dict(params)
        adj_tol = p.pop("adj_tol", 1e-12)
        solver = Solver(p.pop("n"), p.pop("L"), float(eps), p.pop("dt"), **p)
        mu, om = solver.init_guess(phi0)
        p0 = phi0.detach().clone()
        state = (p0, p0.clone(), mu, om)
        ckpts = {}
        for seg in range(0, steps, ckpt_every):
            ckpts[seg] = tuple(t.clone() for t in state)
            phis, mu, om = run_segment(solver, state, min(ckpt_every, steps - seg))
            state = (phis[-2], phis[-1], mu, om)
        ctx.solver, ctx.ckpts, ctx.steps, ctx.every, ctx.adj_tol = solver, ckpts, steps, ckpt_every, adj_tol
        ctx.eps_shape = eps.shape
        ctx.eps_device = eps.device
        return state[1]

    @staticmethod
    def backward(ctx, grad_out):
        s, steps, every = ctx.solver, ctx.steps, ctx.every
        gnext = grad_out.contiguous().clone()        # d/dphi^{k+1}
        gcur = torch.zeros_like(gnext)               # d/dphi^k
        geps = torch.zeros(1, dtype=torch.float64, device=gnext.device)
        for seg in reversed(range(0, steps, every)):
            end = min(seg + every, steps)
            phis, _, _ = run_segment(s, ctx.ckpts[seg], end - seg)   # phis[i] = phi^{seg - 1 + i}
            for k in range(end - 1, seg - 1, -1):
                i = k - seg + 1                      # phis[i] = phi^k
                gprev = torch.zeros_like(gnext)
                if k == 0:                           # phi^{-1} is phi^0: both slots feed gcur
                    s.adjoint_step(phis[i - 1], phis[i], phis[i + 1], gnext, gcur, gcur, geps,
                                   adj_tol=ctx.adj_tol)
                else:
                    s.adjoint_step(phis[i - 1], phis[i], phis[i + 1], gnext, gcur, gprev, geps,
                                   adj_tol=ctx.adj_tol)
                gnext, gcur = gcur, gprev
        grad_eps = geps.reshape(ctx.eps_shape).to(ctx.eps_device)
        return gnext, grad_eps, None, None, None


def rollout(phi0, eps, params, steps, ckpt_every=5):
    return PFCRollout.apply(phi0, eps, params, steps, ckpt_every)
