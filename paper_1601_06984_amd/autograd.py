"""torch.autograd front end of the multilevel run and its hand-written
adjoint, with checkpointing every K coarse steps.

Forward: create a simulation with tau0 and the inflow velocity, initialise
every level from (rho, u, S), run n coarse steps saving the state every K
steps, and return the objective (kinetic energy or the x force).

Backward: seed the adjoint from the final state; for each K-step segment,
last first, restore its checkpoint and reverse the segment's coarse steps
last first; finally reverse the initialisation.  Inside a segment the start
states of the coarse steps are recomputed from the segment checkpoint.  With
no snapshot limit all K of them are kept (memory: one checkpoint per
segment plus K states, recompute: K - 1 steps).  With a limit of s extra
states, the segment is reversed by recursive bisection: advance to the
middle, keep that state, reverse the second half, then the first half
(memory: at most s + 1 states, recompute: O(K log K) steps), as binomial
checkpointing does when the step states do not fit.
"""
from __future__ import annotations

import torch

from . import _lib
from .api import Sim


class MultilevelLBMFunction(torch.autograd.Function):
    """J = apply(spec, tau0, u_in, *u0) with

    spec   dict: plan, precision, rho (list per level), S (list or None),
           n_steps, checkpoint_every, objective ('ke' | 'drag_x'),
           max_snapshots (None: keep every step state of a segment;
           "auto": as many as the free device memory holds)
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
        ctx.max_snapshots = spec.get("max_snapshots")
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
            reverse_steps(sim, ctx.ckpts[start], end - start, ctx.max_snapshots)
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


def snapshot_budget(sim, reserve=0.05):
    """Number of extra step states the free device memory holds, keeping
    `reserve` of the device's memory free."""
    free, total = torch.cuda.mem_get_info(sim.device)
    room = free - int(reserve * total)
    return max(0, room // max(1, sim.checkpoint_bytes()))


def reverse_steps(sim, start_ckpt, n, max_snapshots=None):
    """Reverse n coarse steps whose first starts from the state in
    `start_ckpt`; lambda holds the adjoint of the state after the n steps.
    Keeps at most `max_snapshots` extra states alive (None: no limit;
    "auto": snapshot_budget at the start)."""
    if n <= 0:
        return
    if max_snapshots == "auto":
        max_snapshots = snapshot_budget(sim)
    if n == 1:
        sim.adjoint_step(start_ckpt)
        return
    if max_snapshots is None or max_snapshots >= n - 1:
        sim.load_checkpoint(start_ckpt)
        states = [start_ckpt]
        for _ in range(n - 1):
            sim.step(1)
            states.append(sim.save_checkpoint())
        for st in reversed(states):
            sim.adjoint_step(st)
        return
    if max_snapshots < 1:
        # no room for a state: recompute from the start for every step
        for i in reversed(range(n)):
            sim.load_checkpoint(start_ckpt)
            if i:
                sim.step(i)
                st = sim.save_checkpoint()
                sim.adjoint_step(st)
                del st
            else:
                sim.adjoint_step(start_ckpt)
        return
    m = n // 2
    sim.load_checkpoint(start_ckpt)
    sim.step(m)
    mid = sim.save_checkpoint()
    reverse_steps(sim, mid, n - m, max_snapshots - 1)
    del mid
    reverse_steps(sim, start_ckpt, m, max_snapshots)


def objective(plan, rho, u0, tau0, n_steps, *, S=None, u_in=None, precision="f32",
              checkpoint_every=None, objective="ke", max_snapshots="auto"):
    """Differentiable objective J(u0, tau0[, u_in]) of a multilevel run.
    max_snapshots: extra step states kept while reversing a segment ("auto":
    as many as the free device memory holds; None: all of them)."""
    spec = dict(plan=plan, precision=precision, rho=rho, S=S, n_steps=n_steps,
                checkpoint_every=checkpoint_every or n_steps, objective=objective,
                max_snapshots=max_snapshots)
    return MultilevelLBMFunction.apply(spec, tau0, u_in, *u0)
