"""Element integrals of the Q1-RT0-P0 discretization (oracle; test infra only).

Appendix A (eq. MFE_matrix, MHFE_matrix) defines, per hexahedron T,

* [A_uu]_ij = (sym grad eta_i, C_dr : sym grad eta_j)_T   (Q1 vector basis)
* [A_up]_ij = -(div eta_i, b chi_j)_T                       (chi_j: P0 indicator)
* [A_ww]_ij = (phi_i, mu kappa^-1 phi_j)_T                  (RT0 basis of T)

Quadrature: 2x2x2 Gauss-Legendre on the trilinear map (the paper does not
state a rule; with it the coupling integral of a Q1 gradient is exact on
trilinear hexahedra and the RT0 mass is exact on parallelepipeds).

RT0 basis on the reference cube [-1,1]^3, one function per face, normalised
to unit outward flux through its own face: for axis d, the +d face function is
(1+xi_d)/8 e_d and the -d face function is -(1-xi_d)/8 e_d; mapped by the
contravariant Piola transform phi = J phi_hat / det J.
"""
from __future__ import annotations

import numpy as np

_G = 1.0 / np.sqrt(3.0)
GAUSS_1D = (-_G, _G)
GAUSS_3D = [(x, y, z) for z in GAUSS_1D for y in GAUSS_1D for x in GAUSS_1D]  # weights 1
GAUSS_2D = [(x, y) for y in GAUSS_1D for x in GAUSS_1D]

# reference node signs s_a in {-1,+1}^3, local node a at offset (a&1, (a>>1)&1, (a>>2)&1)
NODE_SIGNS = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                       for a in range(8)], dtype=np.float64)


def lame(E, nu):
    """Lame parameters of an isotropic drained elasticity tensor (Sec. 1)."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    G = E / (2.0 * (1.0 + nu))
    return lam, G


def shape_ref(xi):
    """Trilinear shape functions N_a and reference gradients dN_a/dxi (8,), (8,3)."""
    xi = np.asarray(xi, dtype=np.float64)
    t = 1.0 + NODE_SIGNS * xi[None, :]           # (8,3)
    N = t.prod(axis=1) / 8.0
    dN = np.empty((8, 3))
    dN[:, 0] = NODE_SIGNS[:, 0] * t[:, 1] * t[:, 2] / 8.0
    dN[:, 1] = NODE_SIGNS[:, 1] * t[:, 0] * t[:, 2] / 8.0
    dN[:, 2] = NODE_SIGNS[:, 2] * t[:, 0] * t[:, 1] / 8.0
    return N, dN


def jacobian(X, dNref):
    """J[c, i, j] = d x_i / d xi_j for cells X (nc,8,3)."""
    return np.einsum("cai,aj->cij", X, dNref)


def elasticity_matrix(lam, G):
    """6x6 Voigt matrix (xx, yy, zz, yz, xz, xy; engineering shears), per cell."""
    lam = np.atleast_1d(lam)
    G = np.atleast_1d(G)
    D = np.zeros((lam.size, 6, 6))
    for r in range(3):
        for s in range(3):
            D[:, r, s] = lam
        D[:, r, r] += 2.0 * G
    for r in range(3, 6):
        D[:, r, r] = G
    return D


def strain_matrix(dNx):
    """B (nc,6,24) from physical shape gradients dNx (nc,8,3)."""
    nc = dNx.shape[0]
    B = np.zeros((nc, 6, 24))
    for a in range(8):
        gx, gy, gz = dNx[:, a, 0], dNx[:, a, 1], dNx[:, a, 2]
        B[:, 0, 3 * a + 0] = gx
        B[:, 1, 3 * a + 1] = gy
        B[:, 2, 3 * a + 2] = gz
        B[:, 3, 3 * a + 1] = gz
        B[:, 3, 3 * a + 2] = gy
        B[:, 4, 3 * a + 0] = gz
        B[:, 4, 3 * a + 2] = gx
        B[:, 5, 3 * a + 0] = gy
        B[:, 5, 3 * a + 1] = gx
    return B


def q1_element(X, E, nu, biot):
    """Q1 stiffness K_T (nc,24,24), coupling column a_T = [A_up]_{:,T} (nc,24)
    and cell volumes |T| (nc,), Appendix A eq. MFE_matrix.

    Local dof order 3*a + c (node a, component c).  Raises ValueError on a
    non-positive Jacobian determinant (inverted hexahedron)."""
    X = np.asarray(X, dtype=np.float64)
    nc = X.shape[0]
    lam, G = lame(np.broadcast_to(E, (nc,)), nu)
    D = elasticity_matrix(lam, G)
    K = np.zeros((nc, 24, 24))
    a = np.zeros((nc, 24))
    vol = np.zeros(nc)
    for q in GAUSS_3D:
        _, dNr = shape_ref(q)
        J = jacobian(X, dNr)
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0.0):
            raise ValueError("non-positive Jacobian determinant")
        Jinv = np.linalg.inv(J)
        dNx = np.einsum("aj,cji->cai", dNr, Jinv)     # dN_a/dx_i
        B = strain_matrix(dNx)
        K += np.matmul(np.transpose(B, (0, 2, 1)), np.matmul(D, B)) * detJ[:, None, None]   # B^T D B
        a += -biot * dNx.reshape(nc, 24) * detJ[:, None]
        vol += detJ
    return K, a, vol


def rt0_basis_ref(xi):
    """(6,3) reference RT0 basis values at xi, faces (-x,+x,-y,+y,-z,+z)."""
    phi = np.zeros((6, 3))
    for d in range(3):
        phi[2 * d + 0, d] = -(1.0 - xi[d]) / 8.0
        phi[2 * d + 1, d] = (1.0 + xi[d]) / 8.0
    return phi


def rt0_mass(X, kappa, mu):
    """RT0 element mass M_T (nc,6,6) = (phi_i, mu kappa^-1 phi_j)_T with the
    Piola-mapped, flux-normalised basis; kappa (nc,3) diagonal in global axes."""
    X = np.asarray(X, dtype=np.float64)
    nc = X.shape[0]
    kinv = mu / np.asarray(kappa, dtype=np.float64)
    M = np.zeros((nc, 6, 6))
    for q in GAUSS_3D:
        _, dNr = shape_ref(q)
        J = jacobian(X, dNr)
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0.0):
            raise ValueError("non-positive Jacobian determinant")
        Jphi = np.einsum("cij,fj->cfi", J, rt0_basis_ref(q))
        M += np.einsum("cfi,ci,cgi->cfg", Jphi, kinv, Jphi) / detJ[:, None, None]
    return M


def top_traction(Xface, t):
    """Consistent nodal loads of a traction t (3,) on a bilinear quadrilateral
    face with nodes Xface (nf,4,3) ordered (0,0),(1,0),(0,1),(1,1):
    integral of N_a t dS with 2x2 Gauss.  Returns (nf,4,3)."""
    Xface = np.asarray(Xface, dtype=np.float64)
    s = np.array([[-1, -1], [1, -1], [-1, 1], [1, 1]], dtype=np.float64)
    out = np.zeros(Xface.shape)
    for (x, y) in GAUSS_2D:
        N = (1 + s[:, 0] * x) * (1 + s[:, 1] * y) / 4.0
        dNx = s[:, 0] * (1 + s[:, 1] * y) / 4.0
        dNy = s[:, 1] * (1 + s[:, 0] * x) / 4.0
        tx = np.einsum("a,fai->fi", dNx, Xface)
        ty = np.einsum("a,fai->fi", dNy, Xface)
        dS = np.linalg.norm(np.cross(tx, ty), axis=1)
        out += N[None, :, None] * np.asarray(t)[None, None, :] * dS[:, None, None]
    return out
