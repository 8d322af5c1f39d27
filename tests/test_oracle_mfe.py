"""Pins of the oracle's non-hybridized mixed formulation (CPU only).

Checks against: the algebraic equivalence of the mixed and the mixed hybrid
formulations (same u and p, face fluxes equal to the oriented cell fluxes of
the hybrid solution) on uniform, perturbed and cantilever grids, with and
without stabilization and over two steps; symmetry and definiteness of A_qq;
the discrete divergence of the oriented face basis (one +1 and one -1 per
interior face); the sparsity statement for C~_p in Sec. 5; and FGMRES with the
block triangular preconditioner M_I^(m) against the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.mfe import (BtpPrec, assemble_mfe, build_mfe_system, cp_tilde, face_signs, lumped_aqq,
                        masked_mfe_blocks, solve_mfe_step)
from oracle.solve import fgmres, solve_step
from synth import Problem, perturbed_coords, uniform_coords


def _prob(nx, ny, nz, seed=3, perturb=False, bc="column", **kw):
    rng = np.random.default_rng(seed)
    nc = nx * ny * nz
    coords = perturbed_coords(nx, ny, nz, seed + 1) if perturb else uniform_coords(nx, ny, nz)
    args = dict(nu=0.3, S_eps=1e-6, dt=1e-2, p_top=0.0)
    args.update(kw)
    return Problem("mfe", nx, ny, nz, coords, 1e4 * np.exp(0.3 * rng.standard_normal(nc)),
                   1e-3 * np.exp(rng.standard_normal((nc, 3))), bc=bc, **args)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check_equivalent(prob, u_prev=None, p_prev=None):
    h = solve_step(prob, u_prev=u_prev, p_prev=p_prev)
    m = solve_mfe_step(prob, u_prev=u_prev, p_prev=p_prev)
    assert _rel(m["u"], h["u"]) < 1e-9
    assert _rel(m["p"], h["p"]) < 1e-9
    K = m["K"]
    F = K.B.mesh.cell_faces
    q_from_w = K.s * h["w"]                          # oriented flux seen from each cell
    scale = np.abs(q_from_w).max()
    assert np.abs(m["q"][F] - q_from_w).max() <= 1e-9 * scale
    return h, m


CASES = {
    "column_uniform_drained": dict(nx=4, ny=2, nz=4, p_top=0.7),
    "column_perturbed": dict(nx=4, ny=2, nz=4, perturb=True, p_top=-0.2, S_eps=0.0),
    "column_unstabilized": dict(nx=3, ny=2, nz=3, stabilize=False),
    "cantilever_undrained": dict(nx=4, ny=2, nz=2, bc="cantilever", dt=1e-5, S_eps=0.0),
    "rollers_perturbed": dict(nx=4, ny=4, nz=2, perturb=True, rollers=True, dt=0.5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_mfe_step_equals_hybrid_step(name):
    kw = dict(CASES[name])
    prob = _prob(kw.pop("nx"), kw.pop("ny"), kw.pop("nz"), **kw)
    _check_equivalent(prob)


def test_mfe_equals_hybrid_on_second_step():
    prob = _prob(4, 2, 2, perturb=True, p_top=0.3)
    h1, m1 = _check_equivalent(prob)
    _check_equivalent(prob, u_prev=h1["u"], p_prev=h1["p"])


def test_aqq_symmetric_positive_definite_and_divergence_of_face_basis():
    prob = _prob(4, 2, 2, perturb=True)
    K = assemble_mfe(prob)
    A = K.A_qq.toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    assert (abs(K.A_pq + K.A_qp.T)).max() == 0
    D = K.A_pq.toarray()                             # (cells, faces): (chi_T, div phi_e)
    nb = np.count_nonzero(D, axis=0)
    interior = nb == 2
    assert np.all((nb == 1) | interior)
    assert np.all(D[:, interior].sum(axis=0) == 0)                 # leaves one cell, enters the other
    assert np.all(np.sort(D[:, interior], axis=0)[[0, -1]] == [[-1.0], [1.0]])
    assert np.array_equal(face_signs(1)[0], [-1, 1, -1, 1, -1, 1])


def test_cp_tilde_pattern_is_that_of_apq_aqp_and_spd():
    prob = _prob(4, 4, 4, perturb=True)
    K = assemble_mfe(prob)
    C = cp_tilde(K)
    P = (abs(K.A_pq) @ abs(K.A_qp)).tocsr()
    Cd, Pd = C.toarray(), P.toarray()
    assert np.all((Cd != 0) <= (Pd != 0))
    assert np.allclose(Cd, Cd.T, rtol=0, atol=1e-12 * np.abs(Cd).max())
    assert np.linalg.eigvalsh(Cd).min() > 0
    # the lumping bounds A_qq from above (spectral equivalence, upper side)
    _, _, _, Aqq, _, _ = masked_mfe_blocks(K)
    L = lumped_aqq(K)
    assert np.linalg.eigvalsh(np.diag(L) - Aqq.toarray()).min() >= -1e-12 * L.max()
    Kb = assemble_mfe(_prob(4, 2, 2))                 # box, diagonal kappa: plain row sums
    _, _, _, Aqb, _, _ = masked_mfe_blocks(Kb)
    assert np.allclose(lumped_aqq(Kb), np.asarray(Aqb.sum(axis=1)).ravel(), rtol=1e-14, atol=0)


@pytest.mark.parametrize("dt", [0.1, 1e-5])
def test_btp_exact_inner_solves_reaches_direct_solution(dt):
    prob = _prob(4, 4, 4, bc="cantilever", dt=dt, S_eps=0.0)
    A, b, K = build_mfe_system(prob)
    x_ref = sp.linalg.splu(A.tocsc()).solve(b)
    P = BtpPrec(K)
    x, its, _ = fgmres(lambda v: A @ v, b, P.apply, rtol=1e-10, restart=200)
    assert its < 80
    assert _rel(x, x_ref) < 1e-7
