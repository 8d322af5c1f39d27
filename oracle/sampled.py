"""Selected rows of the step system, assembled one by one (oracle; test infra).

For problems too large for a full oracle assembly, the rows of the
Dirichlet-treated A_H (eq. stab_A) and of the right-hand side (eq.
MHFE_vector with f~_n of Sec. 2.1, from rest) are formed from the element
integrals of only the cells in each row's support, with the same element
routines and the same stabilization, condensation and Dirichlet conventions
as ``system``: a u-row from the (up to 8) hexahedra around its node, a p-row
from its cell and the cells of its macro-element, a pi-row from the (up to
2) cells sharing the face.  A row computed this way equals the same row of
the full assembly (pinned by a CPU test against ``system.build_system``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .element import lame, q1_element, rt0_mass, top_traction
from .mesh import Mesh


def _cells_around_node(m: Mesh, n):
    i, j, k = n % (m.nx + 1), (n // (m.nx + 1)) % (m.ny + 1), n // ((m.nx + 1) * (m.ny + 1))
    out = []
    for ck in (k - 1, k):
        for cj in (j - 1, j):
            for ci in (i - 1, i):
                if 0 <= ci < m.nx and 0 <= cj < m.ny and 0 <= ck < m.nz:
                    out.append(m.cell_id(ci, cj, ck))
    return out


def _face_cells(m: Mesh, f):
    return m.face_cells(int(f))


def _macro_cells(m: Mesh, c):
    i, j, k = m.ci[c], m.cj[c], m.ck[c]
    i0, j0, k0 = i - i % 2, j - j % 2, k - k % 2
    return [m.cell_id(i0 + (a & 1), j0 + ((a >> 1) & 1), k0 + ((a >> 2) & 1)) for a in range(8)]


def system_rows(prob, rows, dt=None):
    """Rows of the Dirichlet-treated A_H (scipy CSR, len(rows) x N) and of b,
    for one step from rest.  ``rows`` index the system vector [u; p; pi]."""
    from .system import dirichlet_sets
    m = Mesh(prob.nx, prob.ny, prob.nz, prob.coords)
    dt = prob.dt if dt is None else dt
    n_u, n_p, n_pi = 3 * m.n_nodes, m.n_cells, m.n_faces
    N = n_u + n_p + n_pi
    rows = np.asarray(rows, dtype=np.int64)
    u_fixed, pi_fixed, pi_bar = dirichlet_sets(prob, m)
    # support cells of every requested row
    need = set()
    for r in rows:
        if r < n_u:
            need.update(_cells_around_node(m, r // 3))
        elif r < n_u + n_p:
            need.update(_macro_cells(m, r - n_u))
        else:
            need.update(_face_cells(m, r - n_u - n_p))
    cells = np.array(sorted(need), dtype=np.int64)
    X = m.coords[m.cell_nodes[cells]]
    Ke, ae, vol = q1_element(X, prob.E[cells], prob.nu, prob.biot)
    Minv = np.linalg.inv(rt0_mass(X, prob.kappa[cells], prob.mu))
    Minv = 0.5 * (Minv + np.transpose(Minv, (0, 2, 1)))
    g = Minv.sum(axis=2)
    alpha = g.sum(axis=1)
    loc = {int(c): q for q, c in enumerate(cells)}
    A = sp.lil_matrix((len(rows), N))
    b = np.zeros(len(rows))
    for ri, r in enumerate(rows):
        r = int(r)
        if r < n_u:
            n, comp = divmod(r, 3)
            for c in _cells_around_node(m, n):
                q = loc[c]
                a = int(np.nonzero(m.cell_nodes[c] == n)[0][0])
                dofs = (3 * m.cell_nodes[c][:, None] + np.arange(3)).ravel()
                for col, v in zip(dofs, Ke[q][3 * a + comp]):
                    A[ri, col] += v
                A[ri, n_u + c] += ae[q][3 * a + comp]
            if m.ck is not None and n // ((m.nx + 1) * (m.ny + 1)) == m.nz:
                ni, nj = n % (m.nx + 1), (n // (m.nx + 1)) % (m.ny + 1)
                for cj in (nj - 1, nj):
                    for ci in (ni - 1, ni):
                        if 0 <= ci < m.nx and 0 <= cj < m.ny:
                            c = m.cell_id(ci, cj, m.nz - 1)
                            Xf = m.coords[m.cell_nodes[c][4:8]][None]
                            la = int(np.nonzero(m.cell_nodes[c][4:8] == n)[0][0])
                            b[ri] += top_traction(Xf, prob.traction)[0, la, comp]
        elif r < n_u + n_p:
            c = r - n_u
            q = loc[c]
            dofs = (3 * m.cell_nodes[c][:, None] + np.arange(3)).ravel()
            for col, v in zip(dofs, ae[q]):
                A[ri, col] += -v
            A[ri, r] += prob.S_eps * vol[q] + dt * alpha[q]
            for e in range(6):
                A[ri, n_u + n_p + m.cell_faces[c][e]] += -dt * g[q][e]
            if prob.stabilize:
                mc = _macro_cells(m, c)
                mv = np.array([vol[loc[t]] for t in mc])
                Eb = float((prob.E[mc] * mv).sum() / mv.sum())
                lam, G = lame(Eb, prob.nu)
                w = (3 * prob.biot) ** 2 / (32 * (lam + 4 * G)) * mv.sum()
                a = mc.index(c)
                for d in range(3):
                    t = mc[a ^ (1 << d)]
                    A[ri, r] += w
                    A[ri, n_u + t] += -w
        else:
            f = r - n_u - n_p
            for c in _face_cells(m, f):
                q = loc[c]
                lf = int(np.nonzero(m.cell_faces[c] == f)[0][0])
                A[ri, n_u + c] += -g[q][lf]
                for e in range(6):
                    A[ri, n_u + n_p + m.cell_faces[c][e]] += Minv[q][lf, e]
    A = A.tocsr()
    # Dirichlet: identity rows; fixed columns lifted to the right-hand side
    fixed = np.concatenate([u_fixed, np.zeros(n_p, bool), pi_fixed])
    xbar = np.concatenate([np.zeros(n_u), np.zeros(n_p), pi_bar])
    b = b - A @ np.where(fixed, xbar, 0.0)
    keep = sp.diags((~fixed).astype(np.float64))
    A = (A @ keep).tolil()
    for ri, r in enumerate(rows):
        if fixed[r]:
            A.rows[ri] = [int(r)]
            A.data[ri] = [1.0]
            b[ri] = xbar[r]
    return A.tocsr(), b
