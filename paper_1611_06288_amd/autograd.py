"""Differentiable rollout of the PFC scheme: torch.autograd.Function whose
backward runs the hand-written adjoint step (``pfc_adjoint_step``).

Forward: ``steps`` time steps of scheme (1.10) from ``phi0`` (bootstrap
phi^{-1} = phi^0), keeping the state (phi^{k-1}, phi^k, mu, omega) every
``ckpt_every`` steps.  Backward: segments are processed last to first; each
is recomputed from its checkpoint (same solver, same tolerance, so the same
trajectory bit for bit) and then walked backwards with one adjoint step per
time step, accumulating d/dphi0 and d/deps.
"""
from __future__ import annotations

import torch

from .solver import Solver


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
        prev, cur = phi0.detach().clone(), phi0.detach().clone()
        ckpts = {}
        for k in range(steps):
            if k % ckpt_every == 0:
                ckpts[k] = (prev.clone(), cur.clone(), mu.clone(), om.clone())
            nxt, _ = solver.step(prev, cur, mu, om)
            prev, cur = cur, nxt
        ctx.solver, ctx.ckpts, ctx.steps, ctx.every, ctx.adj_tol = solver, ckpts, steps, ckpt_every, adj_tol
        ctx.eps_shape = eps.shape
        ctx.eps_device = eps.device
        return cur

    @staticmethod
    def backward(ctx, grad_out):
        s, steps, every = ctx.solver, ctx.steps, ctx.every
        gnext = grad_out.contiguous().clone()        # d/dphi^{k+1}
        gcur = torch.zeros_like(gnext)               # d/dphi^k
        geps = torch.zeros(1, dtype=torch.float64, device=gnext.device)
        for seg in reversed(range(0, steps, every)):
            end = min(seg + every, steps)
            prev, cur, mu, om = (t.clone() for t in ctx.ckpts[seg])
            phis = [prev, cur]                       # phis[i] = phi^{seg - 1 + i}
            for _ in range(seg, end):
                nxt, _ = s.step(phis[-2], phis[-1], mu, om)
                phis.append(nxt.clone())
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
