"""Differentiable poromechanics steps on top of the C ABI.

* ``PoroStep``: one backward-Euler step (u, pi, p) = S(log kappa, log E) as a
  ``torch.autograd.Function``.  Backward solves the transposed block system
  A_H^T lam = dL/dx with FGMRES preconditioned by M^T (``pm_solve_transpose``)
  and accumulates the per-cell gradients (``pm_grad``).
* ``PoroTimeLoop``: N steps with a time-step schedule from rest; returns the
  cell pressures of every step.  The forward pass stores the states only at
  checkpoint steps; backward recomputes each segment from its checkpoint and
  runs the adjoint recursion
      A_n^T lam_n = dL/dx_n + (d b_{n+1} / d x_n)^T lam_{n+1}
  (``pm_rhs_adjoint`` gives the second term), accumulating the gradients of
  every step.

Per-cell parameters: kappa_T = exp(log kappa_T) * aniso_T (aniso: fixed
(n_cells, 3) ratios, ones for isotropic permeability), E_T = exp(log E_T).
All arithmetic runs in the HIP library; this module only sequences calls.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from .solver import PoroSolver


def _materials(logk, logE, aniso):
    kappa = torch.exp(logk.detach().to(torch.float64))[:, None] * aniso
    E = torch.exp(logE.detach().to(torch.float64))
    return E.contiguous(), kappa.contiguous()


class PoroStep(torch.autograd.Function):
    """(u, pi, p) of one step from rest for per-cell log kappa and log E."""

    @staticmethod
    def forward(ctx, logk, logE, solver: PoroSolver, aniso):
        E, kappa = _materials(logk, logE, aniso)
        solver.update_material(E, kappa)
        b = solver.build_rhs()
        u, pi, p, info = solver.solve(b)
        ctx.solver = solver
        ctx.save_for_backward(u, pi, p)
        ctx.info = info
        ctx.state = _solver_state(solver, E, kappa)
        return u, pi, p

    @staticmethod
    def backward(ctx, gu, gpi, gp):
        s: PoroSolver = ctx.solver
        _restore_state(s, ctx.state)
        u, pi, p = ctx.saved_tensors
        dev = u.device
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)  # noqa: E731
        g = torch.cat([gu if gu is not None else z(s.n_u), gp if gp is not None else z(s.n_p),
                       gpi if gpi is not None else z(s.n_pi)]).contiguous()
        lu, lpi, lp, _ = s.solve_transpose(g)
        lam = torch.cat([lu, lp, lpi]).contiguous()
        x = torch.cat([u, p, pi]).contiguous()
        dk, dE = s.grad(lam, x)
        return dk, dE, None, None


def poro_step(solver: PoroSolver, logk, logE, aniso: Optional[torch.Tensor] = None):
    if aniso is None:
        aniso = torch.ones(solver.n_p, 3, dtype=torch.float64, device=solver.device)
    return PoroStep.apply(logk, logE, solver, aniso)


class PoroTimeLoop(torch.autograd.Function):
    """Cell pressures (n_steps, n_cells) of a run from rest over ``dts``."""

    @staticmethod
    def forward(ctx, logk, logE, solver: PoroSolver, aniso, dts: Sequence[float], every: int):
        E, kappa = _materials(logk, logE, aniso)
        solver.update_material(E, kappa)
        n_steps = len(dts)
        ps = []
        ckpt = {0: None}            # step index -> state x_{n} before step n+1 (None = rest)
        x_prev = None
        for n in range(n_steps):
            if n % every == 0:
                ckpt[n] = None if x_prev is None else x_prev.clone()
            x_prev = _step(solver, dts[n], x_prev)
            ps.append(solver.split(x_prev)[1].clone())
        ctx.solver, ctx.dts, ctx.every = solver, list(dts), every
        ctx.ckpt = ckpt
        ctx.infos = None
        ctx.state = _solver_state(solver, E, kappa)
        return torch.stack(ps)

    @staticmethod
    def backward(ctx, gP):
        s: PoroSolver = ctx.solver
        _restore_state(s, ctx.state)
        dts, every = ctx.dts, ctx.every
        n_steps = len(dts)
        dev = gP.device
        dk = torch.zeros(s.n_p, dtype=torch.float64, device=dev)
        dE = torch.zeros(s.n_p, dtype=torch.float64, device=dev)
        lam_next = None
        starts = list(range(0, n_steps, every))
        for c0 in reversed(starts):
            c1 = min(c0 + every, n_steps)
            # recompute the segment's states from its checkpoint
            states = [ctx.ckpt[c0]]
            x = ctx.ckpt[c0]
            for n in range(c0, c1):
                x = _step(s, dts[n], x)
                states.append(x)
            for n in reversed(range(c0, c1)):
                x_n = states[n - c0 + 1]
                x_prev = states[n - c0]
                c = torch.zeros(s.N, dtype=torch.float64, device=dev)
                c[s.n_u:s.n_u + s.n_p] = gP[n].to(torch.float64)
                if lam_next is not None:
                    s.rhs_adjoint(lam_next, c)   # independent of dt
                s.set_dt(dts[n])
                lu, lpi, lp, _ = s.solve_transpose(c)
                lam = torch.cat([lu, lp, lpi]).contiguous()
                p_prev = None if x_prev is None else s.split(x_prev)[1].contiguous()
                s.grad(lam, x_n.contiguous(), p_prev, dk, dE)
                lam_next = lam
        return dk, dE, None, None, None, None


def _solver_state(s: PoroSolver, E, kappa):
    """What the backward pass needs the solver to hold: the forward pass's
    material fields (and the version the solver had right after setting
    them) and its time step."""
    return dict(version=s.material_version, E=E, kappa=kappa, dt=s.dt)


def _restore_state(s: PoroSolver, st):
    """Re-apply the forward pass's material and time step when another
    forward pass, update_material or set_dt has changed the solver since."""
    if s.material_version != st["version"]:
        s.update_material(st["E"], st["kappa"])
        st["version"] = s.material_version
    s.set_dt(st["dt"])


def _step(s: PoroSolver, dt: float, x_prev: Optional[torch.Tensor]) -> torch.Tensor:
    s.set_dt(dt)
    if x_prev is None:
        b = s.build_rhs()
    else:
        u, p, _ = s.split(x_prev)
        b = s.build_rhs(u.contiguous(), p.contiguous())
    u, pi, p, _ = s.solve(b)
    return torch.cat([u, p, pi])


def time_loop(solver: PoroSolver, logk, logE, dts, every: int = 5, aniso: Optional[torch.Tensor] = None):
    if aniso is None:
        aniso = torch.ones(solver.n_p, 3, dtype=torch.float64, device=solver.device)
    return PoroTimeLoop.apply(logk, logE, solver, aniso, list(dts), int(every))
