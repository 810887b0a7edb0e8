"""Receiver misfit as a differentiable function of the per-cell materials.

`misfit(rho, a, b, problem)` returns J (a 0-d float64 tensor) and back-propagates dJ/drho, dJ/da,
dJ/db computed by the discrete adjoint of the ERK stepping (hho_adjoint_step): a = c (fluid) or
lambda (solid), b = mu (solid; its gradient is 0 on fluid cells).  Every forward call builds an
engine for the given materials on the GPU, runs the forward sweep with checkpoints and the
reverse sweep, and keeps the gradient for the backward pass.  Only argument marshalling happens
here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from .hho import Engine


@dataclass
class MisfitProblem:
    """Everything but the materials: mesh topology and media, discretisation, shots, receivers,
    observed data d_obs[n_shots][n_steps][n_rec][2], time window and checkpoint spacing."""
    mesh: dict
    k: int
    dt: float
    n_steps: int
    rec_xy: np.ndarray
    rec_field: np.ndarray
    d_obs: np.ndarray
    sources: list = field(default_factory=list)   # per shot: (xy, dir, f0, t0, amp)
    states: list = field(default_factory=list)    # per shot: initial state (external layout) or None
    t0: float = 0.0
    rk_stages: int = 4
    dtype: str = "f64"
    ckpt_every: int = 0
    eta_f: float = 0.8
    eta_s: float = 1.5
    stab_speed: int = 1

    @property
    def n_shots(self):
        return max(1, len(self.sources), len(self.states))


def _engine(problem: MisfitProblem, rho, a, b):
    mesh = dict(problem.mesh)
    mesh["rho"], mesh["a"], mesh["b"] = rho, a, b
    e = Engine(mesh, problem.k, rk_stages=problem.rk_stages, eta_f=problem.eta_f, eta_s=problem.eta_s,
               stab_speed=problem.stab_speed, dtype=problem.dtype, n_shots=problem.n_shots)
    for sh, src in enumerate(problem.sources):
        if src is not None:
            e.set_sources(sh, *src)
    for sh, U0 in enumerate(problem.states):
        if U0 is not None:
            e.set_state(U0, shot=sh)
    e.set_receivers(problem.rec_xy, problem.rec_field)
    return e


class MisfitFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, a, b, problem):
        as_np = [np.ascontiguousarray(t.detach().to("cpu", torch.float64).numpy()) for t in (rho, a, b)]
        e = _engine(problem, *as_np)
        try:
            J, grad = e.adjoint(problem.t0, problem.dt, problem.n_steps, problem.d_obs, problem.ckpt_every)
        finally:
            e.close()
        g = torch.from_numpy(grad)
        ctx.save_for_backward(g[:, 0].to(rho.device), g[:, 1].to(a.device), g[:, 2].to(b.device))
        return torch.tensor(J, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, gJ):
        g_rho, g_a, g_b = ctx.saved_tensors
        return gJ * g_rho, gJ * g_a, gJ * g_b, None


def misfit(rho: torch.Tensor, a: torch.Tensor, b: torch.Tensor, problem: MisfitProblem) -> torch.Tensor:
    return MisfitFunction.apply(rho, a, b, problem)
