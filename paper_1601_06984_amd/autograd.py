"""torch.autograd front end of the multilevel run and its hand-written
adjoint, with checkpointing every K coarse steps.

Forward: create a simulation with tau0 and the inflow velocity, initialise
every level from (rho, u, S), run n coarse steps saving the state every K
steps, and return the objective (kinetic energy or the x force).

Backward: seed the adjoint from the final state; for each K-step segment,
last first, restore its checkpoint, recompute the segment forward keeping
the start state of every coarse step, and reverse those steps last first;
finally reverse the initialisation.  Memory: one checkpoint per segment
plus K step states inside the segment being reversed.
"""
from __future__ import annotations

import torch

from . import _lib
from .api import Sim


class MultilevelLBMFunction(torch.autograd.Function):
    """J = apply(spec, tau0, u_in, *u0) with

    spec   dict: plan, precision, rho (list per level), S (list or None),
           n_steps, checkpoint_every, objective ('ke' | 'drag_x')
    tau0   0-dim float64 tensor (coarsest-level relaxation time)
    u_in   (d,) float64 tensor (EQ-face velocity) or None
    u0     per-level (d, n_fluid) float64 device tensors (initial velocity)
    """

    @staticmethod
    def forward(ctx, spec, tau0, u_in, *u0):
        plan = spec["plan"]
        n_steps = int(spec["n_steps"])
        K = max(1, int(spec.get("checkpoint_every", n_steps)))
        objective = spec.get("objective", "ke")
        uin = None if u_in is None else u_in.detach().cpu().double().tolist()
        sim = Sim(plan, spec.get("precision", "f32"), float(tau0), u_in=uin)
        rho, S = spec["rho"], spec.get("S")
        u0 = [u.detach().contiguous() for u in u0]
        for k in range(plan.n_levels):
            sim.init(k, rho[k], u0[k], None if S is None else S[k])
        sim.fill_ghosts()
        ckpts = {}
        t = 0
        while t < n_steps:
            ckpts[t] = sim.save_checkpoint()
            m = min(K, n_steps - t)
            sim.step(m)
            t += m
        mask = _lib.DIAG_KE if objective == "ke" else _lib.DIAG_FORCE
        J = sim.diagnostics(mask)[0].clone()
        ctx.sim, ctx.ckpts, ctx.K, ctx.n_steps = sim, ckpts, K, n_steps
        ctx.objective, ctx.rho, ctx.S, ctx.u0 = objective, rho, S, u0
        ctx.has_uin = u_in is not None
        ctx.tau_meta = (tau0.dtype, tau0.device)
        ctx.uin_meta = (u_in.dtype, u_in.device) if u_in is not None else None
        return J

    @staticmethod
    def backward(ctx, gJ):
        sim = ctx.sim
        if not hasattr(sim, "adj_workspace"):
            sim.adjoint_attach()
        sim.adjoint_seed(ctx.objective)
        for start in sorted(ctx.ckpts, reverse=True):
            end = min(start + ctx.K, ctx.n_steps)
            sim.load_checkpoint(ctx.ckpts[start])
            states = []
            for _ in range(start, end):
                states.append(sim.save_checkpoint())
                sim.step(1)
            for st in reversed(states):
                sim.adjoint_step(st)
        n = sim.plan.n_levels
        du = sim.adjoint_init(ctx.rho, ctx.u0,
                              None if ctx.S is None else ctx.S)
        dtau, _, duin = sim.adjoint_params()
        g = float(gJ)
        d_tau = torch.tensor(g * dtau, dtype=ctx.tau_meta[0], device=ctx.tau_meta[1])
        d_uin = None
        if ctx.has_uin:
            d_uin = torch.tensor([g * v for v in duin[:sim.plan.d]], dtype=ctx.uin_meta[0],
                                 device=ctx.uin_meta[1])
        grads = [g * du[k] for k in range(n)]
        return (None, d_tau, d_uin, *grads)


def objective(plan, rho, u0, tau0, n_steps, *, S=None, u_in=None, precision="f32",
              checkpoint_every=None, objective="ke"):
    """Differentiable objective J(u0, tau0[, u_in]) of a multilevel run."""
    spec = dict(plan=plan, precision=precision, rho=rho, S=S, n_steps=n_steps,
                checkpoint_every=checkpoint_every or n_steps, objective=objective)
    return MultilevelLBMFunction.apply(spec, tau0, u_in, *u0)
