"""Solvers and post-processing of the MHFE step (oracle; test infra only).

* ``direct_solve``   the step result is the exact solution of A_H x = b
                     (eq. stab_A); here by sparse LU (SuperLU, COLAMD).
* ``bp_tilde``       B~_p = A_pp + diag(A_stab) + diag(A_up^T diag(A_uu)^-1 A_up)
                     with A_pp the condensed diagonal S|T| + dt*alpha_T
                     (eq. app_Bp and the explicit form stated for M_I^(h); the
                     printed A_pp there is read as the condensed diagonal, since
                     eq. app_Bp keeps the -dt A_pw A_ww^-1 A_wp term).
* ``cpi_tilde``      C~_pi = A_pipi - dt A_pip B~_p^-1 A_ppi (Sec. 4).
* ``BlockPrec``      z = M^-1 r for the block upper triangular M of eq.
                     hybridPrec by back substitution pi -> p -> u; inner inverses
                     exact (variant M_I^(h)); ``transpose`` applies M^-T.
* ``fgmres``         right-preconditioned flexible GMRES, zero initial guess,
                     modified Gram-Schmidt, restart m, stop on the true
                     2-norm residual reduction (Sec. 5 solver settings).
* ``reconstruct_w``  w_T = M_T^-1 (p_T 1 - pi_T), the cell-based velocity
                     reconstruction of Sec. 2.2.
* ``mass_residual``  per-cell continuity residual of the step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .system import Blocks, build_system, split


def direct_solve(A: sp.csr_matrix, b: np.ndarray, transpose=False) -> np.ndarray:
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    return lu.solve(b, trans="T" if transpose else "N")


def masked_blocks(B: Blocks):
    """Blocks with Dirichlet rows/cols treated (identity diagonal blocks)."""
    fu = B.u_fixed.astype(np.float64)
    fpi = B.pi_fixed.astype(np.float64)
    ku, kpi = sp.diags(1.0 - fu), sp.diags(1.0 - fpi)
    Auu = (ku @ B.A_uu @ ku + sp.diags(fu)).tocsr()
    Aup = (ku @ B.A_up).tocsr()
    Apu = (B.A_pu @ ku).tocsr()
    Appi = (B.A_ppi @ kpi).tocsr()
    Apip = (kpi @ B.A_pip).tocsr()
    Apipi = (kpi @ B.A_pipi @ kpi + sp.diags(fpi)).tocsr()
    return Auu, Aup, Apu, Appi, Apip, Apipi


def bp_tilde(B: Blocks) -> np.ndarray:
    Auu, Aup, _, _, _, _ = masked_blocks(B)
    d = Auu.diagonal()
    free = ~B.u_fixed
    Aup_f = Aup[np.nonzero(free)[0]]
    fs = np.asarray(Aup_f.multiply(Aup_f).T @ (1.0 / d[free])).ravel()
    return B.App_bar.diagonal() + B.A_stab.diagonal() + fs


def cpi_tilde(B: Blocks, bp=None) -> sp.csr_matrix:
    bp = bp_tilde(B) if bp is None else bp
    _, _, _, Appi, Apip, Apipi = masked_blocks(B)
    C = Apipi - B.dt * (Apip @ sp.diags(1.0 / bp) @ Appi)
    return C.tocsr()


class BlockPrec:
    """M^-1 of eq. hybridPrec with exact inner solves (M_I^(h))."""

    def __init__(self, B: Blocks):
        self.B = B
        self.Auu, self.Aup, _, self.Appi, _, _ = masked_blocks(B)
        self.bp = bp_tilde(B)
        self.C = cpi_tilde(B, self.bp)
        self.lu_u = spla.splu(self.Auu.tocsc())
        self.lu_c = spla.splu(self.C.tocsc())

    def apply(self, r):
        B = self.B
        ru, rp, rpi = split(B, r)
        zpi = self.lu_c.solve(rpi)
        zp = (rp - B.dt * (self.Appi @ zpi)) / self.bp
        zu = self.lu_u.solve(ru - self.Aup @ zp)
        return np.concatenate([zu, zp, zpi])

    def apply_transpose(self, r):
        """M^-T: forward substitution u -> p -> pi (M^T is block lower)."""
        B = self.B
        ru, rp, rpi = split(B, r)
        zu = self.lu_u.solve(ru, trans="T")
        zp = (rp - self.Aup.T @ zu) / self.bp
        zpi = self.lu_c.solve(rpi - B.dt * (self.Appi.T @ zp), trans="T")
        return np.concatenate([zu, zp, zpi])


def fgmres(A, b, prec=None, rtol=1e-8, restart=200, max_it=1000):
    """Flexible GMRES (right preconditioning, zero initial guess, MGS).

    ``A`` and ``prec`` are callables.  Stops when ||b - A x||_2 <= rtol ||b||_2
    (estimated by the Givens-rotated Hessenberg residual, then confirmed by
    recomputing the true residual at each restart).  Returns
    (x, iterations, history of relative residual estimates)."""
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist
    its = 0
    M = prec if prec is not None else (lambda v: v)
    while its < max_it:
        r = b - A(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            break
        m = min(restart, max_it - its)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        s = np.zeros(m + 1)
        s[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            s[j + 1] = -sn[j] * s[j]
            s[j] = cs[j] * s[j]
            its += 1
            j_done = j + 1
            hist.append(abs(s[j + 1]) / bnorm)
            if abs(s[j + 1]) <= rtol * bnorm:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), s[:j_done])
        x = x + Z[:j_done].T @ y
        if abs(s[j_done]) <= rtol * bnorm:
            if np.linalg.norm(b - A(x)) <= rtol * bnorm:
                break
    return x, its, hist


def reconstruct_w(B: Blocks, p, pi):
    """Outward face fluxes per cell, w_T = M_T^-1 (p_T 1 - pi_T) (nc,6); pi
    must hold the prescribed values on drained faces."""
    F = B.mesh.cell_faces
    return np.einsum("cij,cj->ci", B.Minv, p[:, None] - pi[F])


def mass_residual(B: Blocks, u, p, pi, u_prev=None, p_prev=None, include_stab=True):
    """Per-cell continuity residual b(div(u - u_prev),1)_T + dt sum_faces w +
    S|T|(p - p_prev) [+ (A_stab (p - p_prev))_T]; zero cell by cell when the
    stabilization term is included."""
    du = u if u_prev is None else u - u_prev
    dp = p if p_prev is None else p - p_prev
    w = reconstruct_w(B, p, pi)
    S = B.App_bar.diagonal() - B.dt * B.alpha
    r = B.A_pu @ du + B.dt * w.sum(axis=1) + S * dp
    if include_stab:
        r = r + B.A_stab @ dp
    return r


def solve_step(prob, dt=None, u_prev=None, p_prev=None, increment_stab=True):
    """Direct solve of one step: returns dict(u, p, pi, w, A, b, B)."""
    A, b, B = build_system(prob, dt, u_prev, p_prev, increment_stab)
    x = direct_solve(A, b)
    u, p, pi = split(B, x)
    return dict(u=u, p=p, pi=pi, w=reconstruct_w(B, p, pi), x=x, A=A, b=b, B=B)
