"""Assembly of the stabilized, condensed MHFE block system (oracle; test infra).

Follows Sec. 2.2 (eq. hybridSys, hmfeSys, A_33H), Sec. 3 (eq. J_def, stab_A)
and Appendix A (eq. MHFE_matrix, MHFE_vector):

* per cell, with M_T the RT0 mass, A_wp^e = -1 (the flux-normalised basis has
  unit divergence integral), A_wpi^e = I (unit flux through its own face),
  A_pw = -A_wp^T, A_piw = -A_wpi^T, static condensation of w gives
    Abar_pp,T = S_eps|T| + dt * 1^T M_T^-1 1          (diagonal)
    A_ppi^e  = -(M_T^-1 1)^T ,  A_pip^e = -(M_T^-1 1),  A_pipi^e = M_T^-1
* A_stab = sum_M beta_M |M| sum_{e in Gamma_M} [[chi_i]]_e [[chi_j]]_e over the
  twelve interior faces of every 2x2x2 macro-element, beta_M =
  (3b)^2 / (32 (lambda_M + 4 G_M)) (3D value of Sec. 3)
* A_H = [[A_uu, A_up, 0], [A_pu, Abar_pp + A_stab, dt A_ppi], [0, A_pip, A_pipi]]
  with A_pu = -A_up^T (eq. stab_A)

Dirichlet dofs (fixed displacements, drained faces) are kept in the system:
their rows and columns are replaced by identity, the column contributions of
the prescribed values are moved to the right-hand side, and the right-hand side
holds the prescribed value there (so the dof count matches table tab:grids).

Readings where the paper is silent (each one is listed in the design doc):
* lambda_M, G_M from the volume-weighted mean of E over the macro-element;
* the stabilization acts on the pressure increment of the step (its term
  A_stab p_{n-1} is added to the right-hand side), which is identical to the
  plain form for a step from rest;
* traction on the top face, bottom displacement fixed, top faces drained, all
  other boundary parts natural (traction-free, no-flow).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .element import lame, q1_element, rt0_mass, top_traction
from .mesh import Mesh


@dataclass
class Blocks:
    mesh: Mesh
    n_u: int
    n_p: int
    n_pi: int
    A_uu: sp.csr_matrix        # raw (no Dirichlet)
    A_up: sp.csr_matrix
    A_pu: sp.csr_matrix
    App_bar: sp.csr_matrix
    A_stab: sp.csr_matrix
    A_ppi: sp.csr_matrix       # without the dt factor
    A_pip: sp.csr_matrix
    A_pipi: sp.csr_matrix
    Minv: np.ndarray           # (nc,6,6)
    g: np.ndarray              # (nc,6)  M^-1 1
    alpha: np.ndarray          # (nc,)   1^T M^-1 1
    vol: np.ndarray            # (nc,)
    Ke: np.ndarray             # (nc,24,24)
    ae: np.ndarray             # (nc,24)
    beta: np.ndarray           # (n_macro,)
    macro: np.ndarray          # (n_macro, 8)
    macro_vol: np.ndarray      # (n_macro,)
    u_fixed: np.ndarray        # bool (n_u,)
    pi_fixed: np.ndarray       # bool (n_pi,)
    pi_bar: np.ndarray         # (n_pi,) prescribed face pressure (0 where free)
    f_u: np.ndarray            # (n_u,) traction load
    dt: float
    E: np.ndarray              # (nc,) Young's modulus


def mesh_of(prob) -> Mesh:
    return Mesh(prob.nx, prob.ny, prob.nz, prob.coords)


def dirichlet_sets(prob, mesh: Mesh):
    """Fixed displacement dofs and drained faces of the problem's BCs."""
    n_u = 3 * mesh.n_nodes
    u_fixed = np.zeros(n_u, dtype=bool)
    pi_fixed = np.zeros(mesh.n_faces, dtype=bool)
    pi_bar = np.zeros(mesh.n_faces)
    if getattr(prob, "bc", "column") == "cantilever":
        i, j, k = mesh.node_ijk()
        for n in np.nonzero(i == 0)[0]:
            u_fixed[3 * n:3 * n + 3] = True
        return u_fixed, pi_fixed, pi_bar
    for n in mesh.bottom_nodes():
        u_fixed[3 * n:3 * n + 3] = True
    if getattr(prob, "rollers", False):
        i, j, k = mesh.node_ijk()
        u_fixed[3 * np.nonzero((i == 0) | (i == mesh.nx))[0] + 0] = True
        u_fixed[3 * np.nonzero((j == 0) | (j == mesh.ny))[0] + 1] = True
    top = mesh.top_faces()
    pi_fixed[top] = True
    pi_bar[top] = prob.p_top
    return u_fixed, pi_fixed, pi_bar


def stabilization(mesh: Mesh, E, nu, biot, vol):
    """A_stab from its definition (eq. J_def): loop over macro-elements and
    over the interior faces of each, adding beta_M |M| [[chi_i]][[chi_j]].

    Returns (A_stab csr, beta (n_macro,), macro cells (n_macro,8), |M|)."""
    macro = mesh.macro_elements()
    E = np.asarray(E, dtype=np.float64)
    mvol = vol[macro].sum(axis=1)
    Ebar = (E[macro] * vol[macro]).sum(axis=1) / mvol
    lam, G = lame(Ebar, nu)
    beta = (3.0 * biot) ** 2 / (32.0 * (lam + 4.0 * G))
    # interior faces of the 2x2x2 patch: pairs of local cells differing in one bit
    pairs = [(a, a ^ (1 << d)) for a in range(8) for d in range(3) if not (a >> d) & 1]
    assert len(pairs) == 12
    rows, cols, vals = [], [], []
    for (a, b) in pairs:
        T1, T2 = macro[:, a], macro[:, b]
        w = beta * mvol
        # jump of chi across the face: +1 on T1, -1 on T2
        for (r, sr) in ((T1, 1.0), (T2, -1.0)):
            for (c, sc) in ((T1, 1.0), (T2, -1.0)):
                rows.append(r)
                cols.append(c)
                vals.append(w * sr * sc)
    n = mesh.n_cells
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    return A, beta, macro, mvol


def assemble_blocks(prob, dt=None) -> Blocks:
    """Element integrals, static condensation and stabilization (no BCs)."""
    mesh = mesh_of(prob)
    dt = prob.dt if dt is None else dt
    X = mesh.cell_coords()
    Ke, ae, vol = q1_element(X, prob.E, prob.nu, prob.biot)
    M = rt0_mass(X, prob.kappa, prob.mu)
    Minv = np.linalg.inv(M)
    Minv = 0.5 * (Minv + np.transpose(Minv, (0, 2, 1)))
    g = Minv.sum(axis=2)
    alpha = g.sum(axis=1)
    nc, nn, nf = mesh.n_cells, mesh.n_nodes, mesh.n_faces
    n_u = 3 * nn
    # A_uu, A_up
    dofs = (3 * mesh.cell_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(nc, 24)
    A_uu = sp.coo_matrix((Ke.ravel(), (np.repeat(dofs, 24, axis=1).ravel(),
                                       np.tile(dofs, (1, 24)).ravel())), shape=(n_u, n_u)).tocsr()
    A_up = sp.coo_matrix((ae.ravel(), (dofs.ravel(), np.repeat(np.arange(nc), 24))),
                         shape=(n_u, nc)).tocsr()
    A_pu = (-A_up.T).tocsr()
    App_bar = sp.diags(prob.S_eps * vol + dt * alpha).tocsr()
    F = mesh.cell_faces
    A_ppi = sp.coo_matrix((-g.ravel(), (np.repeat(np.arange(nc), 6), F.ravel())),
                          shape=(nc, nf)).tocsr()
    A_pip = sp.coo_matrix((-g.ravel(), (F.ravel(), np.repeat(np.arange(nc), 6))),
                          shape=(nf, nc)).tocsr()
    A_pipi = sp.coo_matrix((Minv.ravel(), (np.repeat(F, 6, axis=1).ravel(),
                                           np.tile(F, (1, 6)).ravel())), shape=(nf, nf)).tocsr()
    if prob.stabilize:
        A_stab, beta, macro, mvol = stabilization(mesh, prob.E, prob.nu, prob.biot, vol)
    else:
        A_stab = sp.csr_matrix((nc, nc))
        beta, macro, mvol = np.zeros(0), np.zeros((0, 8), dtype=np.int64), np.zeros(0)
    u_fixed, pi_fixed, pi_bar = dirichlet_sets(prob, mesh)
    # traction on the top face: cells of the top layer, local nodes 4..7
    top = mesh.top_cells()
    Xf = X[top][:, 4:8, :]
    loads = top_traction(Xf, prob.traction)           # (ntop,4,3)
    f_u = np.zeros(n_u)
    np.add.at(f_u, (3 * mesh.cell_nodes[top][:, 4:8, None] + np.arange(3)).ravel(), loads.ravel())
    return Blocks(mesh, n_u, nc, nf, A_uu, A_up, A_pu, App_bar, A_stab, A_ppi, A_pip,
                  A_pipi, Minv, g, alpha, vol, Ke, ae, beta, macro, mvol, u_fixed,
                  pi_fixed, pi_bar, f_u, dt, np.asarray(prob.E, dtype=np.float64).copy())


def system_matrix_raw(B: Blocks) -> sp.csr_matrix:
    """A_H of eq. stab_A in order [u; p; pi], before the Dirichlet treatment."""
    return sp.bmat([[B.A_uu, B.A_up, None],
                    [B.A_pu, B.App_bar + B.A_stab, B.dt * B.A_ppi],
                    [None, B.A_pip, B.A_pipi]], format="csr")


def fixed_mask(B: Blocks):
    return np.concatenate([B.u_fixed, np.zeros(B.n_p, dtype=bool), B.pi_fixed])


def fixed_values(B: Blocks):
    return np.concatenate([np.zeros(B.n_u), np.zeros(B.n_p), B.pi_bar])


def apply_dirichlet(A: sp.csr_matrix, b: np.ndarray, fixed: np.ndarray, xbar: np.ndarray):
    """Identity rows/cols on fixed dofs, lifted right-hand side."""
    b = b - A[:, np.nonzero(fixed)[0]] @ xbar[fixed]
    keep = sp.diags((~fixed).astype(np.float64))
    A = (keep @ A @ keep + sp.diags(fixed.astype(np.float64))).tocsr()
    A.eliminate_zeros()
    b = np.where(fixed, xbar, b)
    return A, b


def rhs_raw(B: Blocks, u_prev=None, p_prev=None, increment_stab=True):
    """Right-hand side before BCs: f_u (traction), f_p = A_pu u_{n-1} +
    S_eps|T| p_{n-1} (+ A_stab p_{n-1}, increment reading) (f~_n of Sec. 2.1,
    no fluid source), f_pi = 0 (no-flow)."""
    fu = B.f_u.copy()
    fp = np.zeros(B.n_p)
    if u_prev is not None:
        fp += B.A_pu @ u_prev
    if p_prev is not None:
        S = B.App_bar.diagonal() - B.dt * B.alpha          # S_eps |T|
        fp += S * p_prev
        if increment_stab:
            fp += B.A_stab @ p_prev
    return np.concatenate([fu, fp, np.zeros(B.n_pi)])


def build_system(prob, dt=None, u_prev=None, p_prev=None, increment_stab=True):
    """(A_H with Dirichlet identity rows, lifted b, Blocks)."""
    B = assemble_blocks(prob, dt)
    A = system_matrix_raw(B)
    b = rhs_raw(B, u_prev, p_prev, increment_stab)
    A, b = apply_dirichlet(A, b, fixed_mask(B), fixed_values(B))
    return A, b, B


def split(B: Blocks, x):
    """x in order [u; p; pi] -> (u, p, pi)."""
    return x[:B.n_u], x[B.n_u:B.n_u + B.n_p], x[B.n_u + B.n_p:]
