"""Pins of the oracle's mesh numbering and element integrals (CPU only).

Each test checks the oracle against something other than itself: the dof
counts printed in table tab:grids, closed forms of the RT0 mass on boxes,
exact reproduction of constant velocities (RT0) and of linear displacements
(Q1), rigid-body kernels, and the total force of a uniform traction.
"""
import os

import numpy as np
import pytest

from oracle.element import q1_element, rt0_mass, rt0_basis_ref, shape_ref, jacobian, \
    top_traction, lame, GAUSS_3D
from oracle.mesh import Mesh
from synth import uniform_coords, perturbed_coords

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _grid_rows():
    rows = []
    for line in open(os.path.join(GOLD, "tab_grids.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _grid_rows())
def test_dof_counts_match_tab_grids(row):
    n, n_u, n_pi, n_p, tot = row
    nn = (n + 1) ** 3
    if n <= 40:
        m = Mesh(n, n, n, uniform_coords(n, n, n))
        nn, nf, nc = m.n_nodes, m.n_faces, m.n_cells
    else:
        nf = 3 * n * n * (n + 1)
        nc = n ** 3
    assert 3 * nn == n_u and nf == n_pi and nc == n_p and 3 * nn + nf + nc == tot


def test_numbering_is_a_bijection():
    m = Mesh(4, 6, 2, uniform_coords(4, 6, 2))
    F = m.cell_faces
    assert np.unique(m.cell_nodes).size == m.n_nodes
    assert np.unique(F).size == m.n_faces
    # every interior face belongs to exactly two cells, boundary faces to one
    cnt = np.bincount(F.ravel(), minlength=m.n_faces)
    bd = m.boundary_faces()
    assert np.all(cnt[bd] == 1)
    mask = np.ones(m.n_faces, bool)
    mask[bd] = False
    assert np.all(cnt[mask] == 2)
    # opposite faces of neighbouring cells coincide
    c = m.cell_id(1, 2, 0)
    assert F[c, 1] == F[m.cell_id(2, 2, 0), 0]
    assert F[c, 3] == F[m.cell_id(1, 3, 0), 2]
    assert F[c, 5] == F[m.cell_id(1, 2, 1), 4]


def _box(h):
    X = np.array([[(a & 1) * h[0], ((a >> 1) & 1) * h[1], ((a >> 2) & 1) * h[2]] for a in range(8)])
    return X[None] + np.array([0.3, -0.2, 1.0])


def test_rt0_box_mass_closed_form():
    h = np.array([0.5, 0.25, 2.0])
    kap = np.array([[2.0, 0.3, 7.0]])
    mu = 1.7
    M = rt0_mass(_box(h), kap, mu)[0]
    A = np.array([h[1] * h[2], h[0] * h[2], h[0] * h[1]])
    ref = np.zeros((6, 6))
    for d in range(3):
        s = mu * h[d] / (kap[0, d] * A[d])
        ref[2 * d:2 * d + 2, 2 * d:2 * d + 2] = s * np.array([[1 / 3, -1 / 6], [-1 / 6, 1 / 3]])
    assert np.allclose(M, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())
    Minv = np.linalg.inv(M)
    for d in range(3):
        s = kap[0, d] * A[d] / (mu * h[d])
        assert np.allclose(Minv[2 * d:2 * d + 2, 2 * d:2 * d + 2], s * np.array([[4, 2], [2, 4]]), rtol=1e-12)


def test_rt0_reproduces_constant_velocity_on_parallelepiped():
    # affine cell: x = x0 + F xi_scaled; the Piola image of RT0 holds constants
    Fm = np.array([[1.0, 0.2, -0.1], [0.15, 0.8, 0.05], [0.0, 0.3, 1.3]])
    X = np.array([[(a & 1), ((a >> 1) & 1), ((a >> 2) & 1)] for a in range(8)], float) @ Fm.T
    X = X[None]
    v = np.array([0.7, -1.1, 0.4])
    # outward flux of v through each face: face normal area vectors of the parallelepiped
    e = Fm.T  # edge vectors e_0, e_1, e_2 (rows)
    area = [np.cross(e[1], e[2]), np.cross(e[2], e[0]), np.cross(e[0], e[1])]
    vol = np.dot(e[0], np.cross(e[1], e[2]))
    assert vol > 0
    w = np.zeros(6)
    for d in range(3):
        w[2 * d + 1] = v @ area[d]
        w[2 * d] = -(v @ area[d])
    for q in [(0.1, -0.5, 0.9), (-1, -1, -1), (1, 0.3, -0.2)]:
        _, dNr = shape_ref(q)
        J = jacobian(X, dNr)[0]
        phi = (J @ rt0_basis_ref(q).T).T / np.linalg.det(J)
        assert np.allclose(w @ phi, v, rtol=1e-13, atol=1e-14)
    # mass: w^T M w = integral of v.(mu kappa^-1) v = mu |v|_K^2 vol
    kap = np.array([[0.5, 2.0, 1.5]])
    M = rt0_mass(X, kap, 1.3)[0]
    assert np.isclose(w @ M @ w, 1.3 * np.sum(v * v / kap[0]) * vol, rtol=1e-13)


def _rigid_modes(X):
    c = X.mean(axis=0)
    R = []
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1
        R.append(t.ravel())
    for w in np.eye(3):
        R.append(np.cross(w, X - c).ravel())
    return np.array(R).T


@pytest.mark.parametrize("perturb", [False, True])
def test_q1_rigid_body_kernel_and_linear_patch(perturb):
    X = perturbed_coords(1, 1, 1, seed=3, amp=0.0)[None] if not perturb else None
    if perturb:
        rng = np.random.default_rng(5)
        X = _box(np.array([1.0, 0.8, 1.2])) + rng.uniform(-0.15, 0.15, (1, 8, 3))
    E, nu, b = 3.0e4, 0.3, 0.9
    K, a, vol = q1_element(X, E, nu, b)
    K, a = K[0], a[0]
    R = _rigid_modes(X[0])
    assert np.abs(K @ R).max() <= 1e-11 * np.abs(K).max()
    # sum over nodes of the coupling column per component is zero (translations)
    assert np.allclose(a.reshape(8, 3).sum(axis=0), 0.0, atol=1e-14)
    # linear field u = G x: energy = |T| eps:C:eps and coupling = -b tr(G)|T|, exact
    Gm = np.array([[0.01, 0.003, -0.002], [0.004, -0.02, 0.001], [0.0, 0.005, 0.015]])
    u = (X[0] @ Gm.T).ravel()
    eps = 0.5 * (Gm + Gm.T)
    lam, G = lame(E, nu)
    dens = lam * np.trace(eps) ** 2 + 2 * G * np.sum(eps * eps)
    assert np.isclose(u @ K @ u, dens * vol[0], rtol=1e-12)
    assert np.isclose(a @ u, -b * np.trace(Gm) * vol[0], rtol=1e-12)
    # volume of the hexahedron by the divergence theorem on its triangulated faces
    assert vol[0] > 0


def test_q1_uniaxial_strain_stress():
    X = _box(np.array([1.0, 1.0, 1.0]))
    E, nu = 1e4, 0.25
    K, _, vol = q1_element(X, E, nu, 1.0)
    eps = 1e-3
    u = np.zeros((8, 3))
    u[:, 2] = eps * X[0][:, 2]
    f = K[0] @ u.ravel()
    lam, G = lame(E, nu)
    # nodal forces on the top nodes sum to sigma_zz * area, with sigma_zz=(lambda+2G) eps
    top = [a for a in range(8) if (a >> 2) & 1]
    assert np.isclose(f.reshape(8, 3)[top, 2].sum(), (lam + 2 * G) * eps, rtol=1e-12)
    # lateral stress sigma_xx = lambda eps on the +x face
    right = [a for a in range(8) if a & 1]
    assert np.isclose(f.reshape(8, 3)[right, 0].sum(), lam * eps, rtol=1e-12)


def test_traction_total_force():
    Xf = np.array([[[0, 0, 1], [0.5, 0, 1], [0, 0.25, 1], [0.5, 0.25, 1]]], float)
    f = top_traction(Xf, (0.0, 0.0, -2.0))
    assert np.isclose(f[..., 2].sum(), -2.0 * 0.125, rtol=1e-14)
    assert np.allclose(f[0, :, 2], -2.0 * 0.125 / 4)


def test_inverted_element_is_rejected():
    X = _box(np.array([1.0, 1.0, 1.0]))
    X[0, [0, 7]] = X[0, [7, 0]]
    with pytest.raises(ValueError):
        q1_element(X, 1.0, 0.25, 1.0)


def test_gauss_rule_has_unit_weights_and_volume():
    X = _box(np.array([0.5, 2.0, 1.5]))
    _, _, vol = q1_element(X, 1.0, 0.25, 1.0)
    assert np.isclose(vol[0], 1.5, rtol=1e-14)
    assert len(GAUSS_3D) == 8
