"""Adjoint of the MHFE step(s) and per-cell gradients (oracle; test infra).

The paper has no adjoint; this restates the plain Lagrangian derivative of
the exact step solution x_n = A_n^-1 b_n(x_{n-1}) (eq. stab_A with the
right-hand side of Sec. 2.1), with Dirichlet dofs held fixed:

* A_n^T lam_n = dL/dx_n + (d b_{n+1} / d x_n)^T lam_{n+1}
  where b_{n+1} depends on x_n through its pressure rows
  A_pu u_n + S_eps|T| p_n + A_stab p_n (increment form of the stabilization);
* dL/dtheta = sum_n -lam_n^T (dA_n/dtheta x_n - d b_n/dtheta), lam restricted
  to rows that are not Dirichlet rows.

Per-cell parameters: theta = log kappa_T (all three diagonal components scaled
together) and log E_T.  The condensed element block of cell T
  K_T = [[dt alpha_T, -dt g_T^T], [-g_T, M_T^-1]]  (rows/cols p_T, faces of T)
is linear in kappa_T, so it is its own log-derivative; the Q1 stiffness is
linear in E_T; beta_M depends on the volume-weighted mean E of its macro-element.
B~_p and C~_pi only shape the preconditioner and carry no gradient.
Pinned by central finite differences of the forward oracle (tests).
"""
from __future__ import annotations

import numpy as np

from .solve import direct_solve
from .system import build_system, split


def _free_lambda(B, lam):
    lu, lp, lpi = split(B, lam)
    lu = np.where(B.u_fixed, 0.0, lu)
    lpi = np.where(B.pi_fixed, 0.0, lpi)
    return lu, lp, lpi


def step_gradients(B, lam, x, p_prev=None):
    """Return (dL/dlogkappa, dL/dlogE) contributions -lam^T dA/dtheta x
    (+ lam^T db/dtheta for the stabilization's right-hand side term)."""
    mesh = B.mesh
    lu, lp, lpi = _free_lambda(B, lam)
    u, p, pi = split(B, x)
    F = mesh.cell_faces
    # kappa: condensed element block
    xl_pi = pi[F]
    ll_pi = lpi[F]
    rows_p = B.dt * B.alpha * p - B.dt * np.einsum("ci,ci->c", B.g, xl_pi)
    rows_pi = -B.g * p[:, None] + np.einsum("cij,cj->ci", B.Minv, xl_pi)
    dk = -(lp * rows_p + np.einsum("ci,ci->c", ll_pi, rows_pi))
    # E: Q1 stiffness (linear in E_T)
    dofs = (3 * mesh.cell_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)
    dE = -np.einsum("ci,cij,cj->c", lu[dofs], B.Ke, u[dofs])
    # E: stabilization coefficient of each macro-element
    if B.macro.shape[0] > 0:
        dp = p if p_prev is None else p - p_prev
        E = B.E
        pairs = [(a, a ^ (1 << d)) for a in range(8) for d in range(3) if not (a >> d) & 1]
        Lq = np.zeros(B.macro.shape[0])          # lam_M^T L_cube dp_M
        for (a, b) in pairs:
            Ta, Tb = B.macro[:, a], B.macro[:, b]
            Lq += (lp[Ta] - lp[Tb]) * (dp[Ta] - dp[Tb])
        wE = E[B.macro] * B.vol[B.macro]
        dbeta = -B.beta[:, None] * wE / wE.sum(axis=1)[:, None]   # d beta_M / d log E_T
        contrib = -(dbeta * (B.macro_vol * Lq)[:, None])
        np.add.at(dE, B.macro.ravel(), contrib.ravel())
    return dk, dE


def loss_obs(B, x, obs):
    """L = sum over observation cells of p_T^2, and dL/dx."""
    u, p, pi = split(B, x)
    g = np.zeros_like(x)
    g[B.n_u + obs] = 2.0 * p[obs]
    return float(np.sum(p[obs] ** 2)), g


def single_step(prob, obs):
    """Forward direct solve, loss, adjoint solve and gradients of one step."""
    A, b, B = build_system(prob)
    x = direct_solve(A, b)
    L, g = loss_obs(B, x, obs)
    lam = direct_solve(A, g, transpose=True)
    dk, dE = step_gradients(B, lam, x)
    return dict(x=x, loss=L, lam=lam, dlogk=dk, dlogE=dE, B=B, A=A)


def multi_step(prob, dts, obs, increment_stab=True):
    """Forward over all steps from rest, loss summed over steps, reverse
    adjoint sweep and gradients (no checkpointing: states kept)."""
    xs, Bs, As = [], [], []
    u_prev = p_prev = None
    for dt in dts:
        A, b, B = build_system(prob, dt, u_prev, p_prev, increment_stab)
        x = direct_solve(A, b)
        xs.append(x)
        Bs.append(B)
        As.append(A)
        u_prev, p_prev, _ = split(B, x)
    L = 0.0
    dk = np.zeros(prob.n_cells)
    dE = np.zeros(prob.n_cells)
    lam_next = None
    for n in reversed(range(len(dts))):
        B, A, x = Bs[n], As[n], xs[n]
        Ln, g = loss_obs(B, x, obs)
        L += Ln
        c = g.copy()
        if lam_next is not None:
            Bn = Bs[n + 1]
            _, lp1, _ = split(Bn, lam_next)
            S = Bn.App_bar.diagonal() - Bn.dt * Bn.alpha
            c[:B.n_u] += -(Bn.A_up @ lp1)
            sp_term = S * lp1
            if increment_stab:
                sp_term = sp_term + Bn.A_stab.T @ lp1
            c[B.n_u:B.n_u + B.n_p] += sp_term
        lam = direct_solve(A, c, transpose=True)
        pprev = None if n == 0 else split(Bs[n - 1], xs[n - 1])[1]
        k_, E_ = step_gradients(B, lam, x, pprev if increment_stab else None)
        dk += k_
        dE += E_
        lam_next = lam
    return dict(xs=xs, loss=L, dlogk=dk, dlogE=dE)


def forward_loss(prob, obs, dts=None, increment_stab=True):
    """Loss of the forward direct solve(s) only (for finite differences)."""
    if dts is None:
        A, b, B = build_system(prob)
        x = direct_solve(A, b)
        return loss_obs(B, x, obs)[0]
    L = 0.0
    u_prev = p_prev = None
    for dt in dts:
        A, b, B = build_system(prob, dt, u_prev, p_prev, increment_stab)
        x = direct_solve(A, b)
        L += loss_obs(B, x, obs)[0]
        u_prev, p_prev, _ = split(B, x)
    return L
