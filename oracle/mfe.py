"""The non-hybridized mixed formulation (MFE) and its block triangular
preconditioner (oracle; test infrastructure only).

Follows Sec. 2.1 (eq. mfeSys), Sec. 3 (the stabilized pressure block
A_pp + A_stab), Appendix A (eq. MFE_matrix, MFE_vector) and Sec. 5 (eq. prec,
variant M_I^(m)).

Unknowns are [u; q; p]: nodal displacements, one Darcy flux per face of the
grid (all faces, as counted in table tab:grids) and one pressure per cell.
The face basis phi_e is oriented by the global +x, +y or +z normal of its
face.  On a cell T it equals s_{T,e} times the cell's outward-normal RT0
basis, with s_{T,e} = -1 on the cell's -x, -y, -z faces and +1 on its +x,
+y, +z faces.  With the flux-normalised basis of the hybrid oracle
(unit divergence integral per outward basis function):

* A_qq = sum_T S_T^T M_T S_T, with M_T the RT0 mass of the cell;
* [A_qp]_{e,T} = -(div phi_e, chi_T)_T = -s_{T,e};  A_pq = -A_qp^T;
* A_pp = diag(S_eps |T|); the pressure block of the stabilized system is
  A_pp + A_stab, with the same A_stab as the hybrid system;
* f_q on a drained face e of cell T is -(phi_e . n, pbar)_e = -s_{T,e} pbar_e
  (the outward normal of the domain there is the cell's outward normal).

Faces on the no-flow boundary carry q = 0 and are kept as identity rows, as
are the fixed displacements.

Hybridization is an algebraic reformulation of the same discrete problem:
the face multiplier pi enforces the flux continuity that MFE builds into its
basis.  The MFE step therefore has the same u and p as the hybrid step, and
q_e = s_{T,e} w_{T,e} for the cell fluxes w reconstructed from the hybrid
solution.  The tests pin this module against the (separately pinned) hybrid
oracle through that identity.

Readings where the paper is silent (listed in the design notes):
* the lumped, spectrally equivalent replacement of A_qq in C~_p is
  L_qq = diag(sum_j |[A_qq]_ij|): positive, L_qq - A_qq is diagonally
  dominant (so A_qq <= L_qq), and on axis-aligned boxes with diagonal kappa,
  where every entry of A_qq in the oriented basis is non-negative, it is the
  plain row-sum lumping.  Plain row sums can be negative on distorted cells,
  where faces of different directions couple with either sign;
* the fixed-stress term of C~_p is diag(A_up^T diag(A_uu)^-1 A_up), the
  same term as in the hybrid B~_p;
* the right-hand side f_p is the one of the hybrid oracle: A_pu u_{n-1} +
  S_eps |T| p_{n-1} (+ A_stab p_{n-1} under the increment reading).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import rt0_mass
from .system import Blocks, apply_dirichlet, assemble_blocks


def face_signs(n_cells: int) -> np.ndarray:
    """s_{T,e} for the six local faces (-x, +x, -y, +y, -z, +z) of every cell."""
    return np.tile(np.array([-1.0, 1.0, -1.0, 1.0, -1.0, 1.0]), (n_cells, 1))


@dataclass
class MfeBlocks:
    B: Blocks                  # hybrid blocks (A_uu, A_up, A_pu, A_stab, BCs, loads)
    n_q: int
    A_qq: sp.csr_matrix
    A_qp: sp.csr_matrix
    A_pq: sp.csr_matrix
    A_pp: sp.csr_matrix        # diag(S_eps |T|)
    s: np.ndarray              # (nc,6) orientation signs
    q_fixed: np.ndarray        # bool (n_q,): no-flow boundary faces
    f_q: np.ndarray            # (n_q,)
    dt: float


def assemble_mfe(prob, dt=None) -> MfeBlocks:
    """Element integrals of eq. MFE_matrix (no Dirichlet treatment)."""
    B = assemble_blocks(prob, dt)
    mesh = B.mesh
    nc, nf = mesh.n_cells, mesh.n_faces
    M = rt0_mass(mesh.cell_coords(), prob.kappa, prob.mu)           # (nc,6,6), outward basis
    s = face_signs(nc)
    F = mesh.cell_faces
    Mg = M * s[:, :, None] * s[:, None, :]
    A_qq = sp.coo_matrix((Mg.ravel(), (np.repeat(F, 6, axis=1).ravel(), np.tile(F, (1, 6)).ravel())),
                         shape=(nf, nf)).tocsr()
    A_qp = sp.coo_matrix(((-s).ravel(), (F.ravel(), np.repeat(np.arange(nc), 6))), shape=(nf, nc)).tocsr()
    A_pq = (-A_qp.T).tocsr()
    S = B.App_bar.diagonal() - B.dt * B.alpha                       # S_eps |T|
    A_pp = sp.diags(S).tocsr()
    ncell_of_face = np.bincount(F.ravel(), minlength=nf)
    boundary = ncell_of_face == 1
    q_fixed = boundary & ~B.pi_fixed
    f_q = np.zeros(nf)
    for c in range(nc):
        for loc in range(6):
            e = F[c, loc]
            if B.pi_fixed[e]:
                f_q[e] -= s[c, loc] * B.pi_bar[e]
    return MfeBlocks(B, nf, A_qq, A_qp, A_pq, A_pp, s, q_fixed, f_q, B.dt)


def mfe_matrix_raw(K: MfeBlocks) -> sp.csr_matrix:
    """A_M of eq. mfeSys with the stabilized pressure block, order [u; q; p]."""
    B = K.B
    return sp.bmat([[B.A_uu, None, B.A_up],
                    [None, K.A_qq, K.A_qp],
                    [B.A_pu, K.dt * K.A_pq, K.A_pp + B.A_stab]], format="csr")


def mfe_fixed_mask(K: MfeBlocks) -> np.ndarray:
    return np.concatenate([K.B.u_fixed, K.q_fixed, np.zeros(K.B.n_p, dtype=bool)])


def mfe_rhs_raw(K: MfeBlocks, u_prev=None, p_prev=None, increment_stab=True) -> np.ndarray:
    """[f_u; f_q; f_p] of eq. MFE_vector (traction, drained-face pressure,
    previous step's volumetric terms; no fluid source)."""
    B = K.B
    fp = np.zeros(B.n_p)
    if u_prev is not None:
        fp += B.A_pu @ u_prev
    if p_prev is not None:
        fp += K.A_pp.diagonal() * p_prev
        if increment_stab:
            fp += B.A_stab @ p_prev
    return np.concatenate([B.f_u, K.f_q, fp])


def build_mfe_system(prob, dt=None, u_prev=None, p_prev=None, increment_stab=True):
    """(A_M with identity rows on fixed u and no-flow q, lifted b, MfeBlocks)."""
    K = assemble_mfe(prob, dt)
    A = mfe_matrix_raw(K)
    b = mfe_rhs_raw(K, u_prev, p_prev, increment_stab)
    fixed = mfe_fixed_mask(K)
    A, b = apply_dirichlet(A, b, fixed, np.zeros(fixed.size))
    return A, b, K


def split_mfe(K: MfeBlocks, x):
    """x in order [u; q; p] -> (u, q, p)."""
    n_u, n_q = K.B.n_u, K.n_q
    return x[:n_u], x[n_u:n_u + n_q], x[n_u + n_q:]


def solve_mfe_step(prob, dt=None, u_prev=None, p_prev=None, increment_stab=True):
    """Direct sparse solve of one MFE step: dict(u, q, p, x, A, b, K)."""
    A, b, K = build_mfe_system(prob, dt, u_prev, p_prev, increment_stab)
    x = spla.splu(A.tocsc(), permc_spec="COLAMD").solve(b)
    u, q, p = split_mfe(K, x)
    return dict(u=u, q=q, p=p, x=x, A=A, b=b, K=K)


def masked_mfe_blocks(K: MfeBlocks):
    """(A_uu, A_up, A_pu, A_qq, A_qp, A_pq) with the fixed rows and columns of
    u and q treated as in the assembled system (identity diagonal blocks)."""
    B = K.B
    fu = B.u_fixed.astype(np.float64)
    fq = K.q_fixed.astype(np.float64)
    ku, kq = sp.diags(1.0 - fu), sp.diags(1.0 - fq)
    Auu = (ku @ B.A_uu @ ku + sp.diags(fu)).tocsr()
    Aup = (ku @ B.A_up).tocsr()
    Apu = (B.A_pu @ ku).tocsr()
    Aqq = (kq @ K.A_qq @ kq + sp.diags(fq)).tocsr()
    Aqp = (kq @ K.A_qp).tocsr()
    Apq = (K.A_pq @ kq).tocsr()
    return Auu, Aup, Apu, Aqq, Aqp, Apq


def lumped_aqq(K: MfeBlocks) -> np.ndarray:
    """Absolute row-sum lumping of the masked A_qq."""
    _, _, _, Aqq, _, _ = masked_mfe_blocks(K)
    return np.asarray(abs(Aqq).sum(axis=1)).ravel()


def cp_tilde(K: MfeBlocks) -> sp.csr_matrix:
    """C~_p = A_stab + A_pp + diag(A_up^T diag(A_uu)^-1 A_up)
    + dt A_qp^T L_qq^-1 A_qp (Sec. 5, the approximation of C_p in eq. prec;
    A_pq = -A_qp^T turns both subtracted products into added ones)."""
    B = K.B
    Auu, Aup, _, _, Aqp, _ = masked_mfe_blocks(K)
    d = Auu.diagonal()
    free = np.nonzero(~B.u_fixed)[0]
    Aup_f = Aup[free]
    fs = np.asarray(Aup_f.multiply(Aup_f).T @ (1.0 / d[free])).ravel()
    L = lumped_aqq(K)
    C = B.A_stab + K.A_pp + sp.diags(fs) + K.dt * (Aqp.T @ sp.diags(1.0 / L) @ Aqp)
    return C.tocsr()


class BtpPrec:
    """M^-1 of eq. prec (block lower triangular) with exact inner solves of
    A_uu, A_qq and C~_p (variant M_I^(m)): z_u = A_uu^-1 r_u,
    z_q = A_qq^-1 r_q, z_p = C~_p^-1 (r_p - A_pu z_u - dt A_pq z_q)."""

    def __init__(self, K: MfeBlocks):
        self.K = K
        Auu, _, self.Apu, Aqq, _, self.Apq = masked_mfe_blocks(K)
        self.C = cp_tilde(K)
        self.lu_u = spla.splu(Auu.tocsc())
        self.lu_q = spla.splu(Aqq.tocsc())
        self.lu_c = spla.splu(self.C.tocsc())

    def apply(self, r):
        K = self.K
        ru, rq, rp = split_mfe(K, r)
        zu = self.lu_u.solve(ru)
        zq = self.lu_q.solve(rq)
        zp = self.lu_c.solve(rp - self.Apu @ zu - K.dt * (self.Apq @ zq))
        return np.concatenate([zu, zq, zp])
