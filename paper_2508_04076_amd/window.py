"""Differentiable fixed-topology windows of the explicit step.

``window(sim, E, u0, v0, n_steps, every, step0)`` runs ``n_steps`` steps of a
:class:`~paper_2508_04076_amd.cem.Simulation` from the state (u0, v0) at step
``step0`` (the load ramp's clock) with the per-tet Young's modulus E and the
crack pass off, and returns (u_n, v_n).  It
is a ``torch.autograd.Function``: the backward is the library's discrete
adjoint of the Newmark update (beta = 0, gamma = 1/2, end of Section 2.2),
which recomputes each checkpoint segment of ``every`` steps and reverses it
step by step on the GPU.  This module only moves arrays between torch and the
library; every step of the computation runs in the library's kernels.

``strain_energy(sim, E, u)`` is the strain energy at displacement u for the
modulus the simulation holds (the E last given to ``window``), differentiable
in E (at fixed u) and u; ``strain_energy(sim, E, window(...)[0])`` is the
end-of-window strain energy, whose gradient in E sums the explicit term and
the window's adjoint.

The time step is an input of the window (set on the simulation), not a
function of E.  Between the forward and the backward the simulation must not
be stepped or modified (the library then refuses the backward).
"""
from __future__ import annotations

import numpy as np
import torch


def _host(t):
    return None if t is None else t.detach().to("cpu", torch.float64).numpy()


class ModulusWindow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, u0, v0, sim, n_steps, every, step0):
        sim.set_modulus(_host(E))
        sim.set_state(_host(u0), _host(v0))
        sim.set_step(step0)
        sim.window_forward(n_steps, every)
        u, v, _ = sim.get_state()
        ctx.sim = sim
        dev = E.device
        return torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gu, gv):
        gu0, gv0, gE = ctx.sim.window_backward(_host(gu), _host(gv))
        dev = gu.device if gu is not None else gv.device
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        return to(gE), to(gu0), to(gv0), None, None, None, None


def window(sim, E, u0, v0, n_steps, every=50, step0=0):
    """(u_n, v_n) after n_steps fixed-topology steps from step step0,
    differentiable in E, u0 and v0."""
    return ModulusWindow.apply(E, u0, v0, sim, int(n_steps), int(every), int(step0))


class StrainEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, u, sim):
        se, gu, gE = sim.strain_energy_grad(_host(u))
        ctx.save_for_backward(torch.from_numpy(gu).to(u.device), torch.from_numpy(gE).to(E.device))
        return torch.tensor(se, dtype=torch.float64, device=u.device)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        gu, gE = ctx.saved_tensors
        return g * gE, g * gu, None


def strain_energy(sim, E, u):
    """1/2 u^T K(E) u with E the modulus the simulation holds (differentiable)."""
    return StrainEnergy.apply(E, u, sim)
