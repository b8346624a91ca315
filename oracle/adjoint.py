"""Reverse pass of the oracle: gradients of an objective after n coarse steps
with respect to the initial velocity field, tau0 and the inflow velocity.

The reverse pass is reverse-mode automatic differentiation of the plain
forward oracle run (torch.autograd), so it is the exact derivative of the
discrete method by definition; it is pinned against central finite
differences of the forward run in the tests.  Runs use ``poison=False``:
missing pull sources hold the rest equilibrium instead of NaN, which changes
no valid value (the NaN-poisoned forward proves that) but keeps 0 * NaN out
of the backward pass.

Objectives (reading taken; they are not in the paper):
* 'ke'      E = 1/2 sum_L V_L sum_fluid rho |u|^2 at the final time;
* 'drag_x'  the x component of the momentum-exchange force (Sec. 2.3).
tau_L follows tau0 through Eq. fneq_scale.
"""
from __future__ import annotations

import numpy as np
import torch

from .solver import OracleSim


def run_objective(mesh, tau0, rho, u, S, n_steps, objective="ke", u_in=None, walls=None):
    sim = OracleSim(mesh, tau0, u_in=u_in, poison=False, walls=walls)
    sim.init(rho, u, S)
    sim.step(n_steps)
    if objective == "ke":
        return sim.kinetic_energy()
    if objective == "drag_x":
        return sim.force()[0]
    raise ValueError(objective)


def gradient(mesh, tau0: float, rho, u, S, n_steps: int, objective="ke",
             u_in=None, walls=None):
    """Returns (J, dJ/dtau0, {L: dJ/du0_L (n_fluid, d)}, dJ/du_in or None)."""
    tau = torch.tensor(float(tau0), dtype=torch.float64, requires_grad=True)
    uu = {L: torch.tensor(np.asarray(u[L]), dtype=torch.float64, requires_grad=True)
          for L in u}
    uin = None
    if u_in is not None:
        uin = torch.tensor(np.asarray(u_in), dtype=torch.float64, requires_grad=True)
    J = run_objective(mesh, tau, rho, uu, S, n_steps, objective, uin, walls)
    inputs = [tau] + [uu[L] for L in sorted(uu)] + ([uin] if uin is not None else [])
    grads = torch.autograd.grad(J, inputs, allow_unused=True)
    g_tau = grads[0]
    g_u = {L: (g if g is not None else torch.zeros_like(uu[L]))
           for L, g in zip(sorted(uu), grads[1:1 + len(uu)])}
    g_in = grads[-1] if uin is not None else None
    return float(J.detach()), float(g_tau), {L: g.numpy() for L, g in g_u.items()}, \
        (g_in.numpy() if g_in is not None else None)


def central_difference(mesh, tau0, rho, u, S, n_steps, objective="ke",
                       du=None, dtau=0.0, duin=None, u_in=None, eps=1e-6, walls=None):
    """(J(x + eps d) - J(x - eps d)) / (2 eps) along the direction
    (du per level, dtau, duin)."""
    def shifted(sign):
        u2 = {L: np.asarray(u[L]) + sign * eps * (du[L] if du is not None else 0.0)
              for L in u}
        uin2 = None
        if u_in is not None:
            uin2 = np.asarray(u_in) + sign * eps * (duin if duin is not None else 0.0)
        with torch.no_grad():
            return float(run_objective(mesh, tau0 + sign * eps * dtau, rho, u2, S,
                                       n_steps, objective, uin2, walls))
    return (shifted(+1) - shifted(-1)) / (2 * eps)
