"""Pins of the oracle's condensed, stabilized system (CPU only).

Checks against: the cube-graph spectrum of the stabilization, the sparsity
inclusion stated for A_stab, the zero-flux identity of the condensed element,
local mass conservation (per cell with the stabilization flux, per
macro-element without it), the spurious pressure modes of Q1-P0 and their
removal, Terzaghi's closed form, the eigenvalue statements of Theorem 1,
Lemma 1, Theorem 2, its remark and Lemma 2, the direct solve against the
preconditioned FGMRES, and the adjoint against central finite differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import terzaghi
from oracle.adjoint import forward_loss, multi_step, single_step
from oracle.element import lame
from oracle.solve import (BlockPrec, bp_tilde, cpi_tilde, direct_solve, fgmres,
                          masked_blocks, mass_residual, reconstruct_w, solve_step)
from oracle.system import assemble_blocks, build_system, split, fixed_mask
from synth import Problem, make_config, uniform_coords


def _small(n=4, **kw):
    nc = n ** 3
    rng = np.random.default_rng(11)
    args = dict(nu=0.25, S_eps=0.0, dt=1e-2)
    args.update(kw)
    return Problem("t", n, n, n, uniform_coords(n, n, n), 1e4 * np.exp(0.3 * rng.standard_normal(nc)),
                   np.repeat((1e-3 * np.exp(rng.standard_normal(nc)))[:, None], 3, 1), **args)


def test_stabilization_spectrum_kernel_and_beta():
    prob = _small(4)
    B = assemble_blocks(prob)
    A = B.A_stab.toarray()
    assert np.allclose(A, A.T)
    for M, beta, mv in zip(B.macro, B.beta, B.macro_vol):
        ev = np.linalg.eigvalsh(A[np.ix_(M, M)]) / (beta * mv)
        assert np.allclose(ev, [0, 2, 2, 2, 4, 4, 4, 6], atol=1e-12)
        lam, G = lame((prob.E[M] * B.vol[M]).sum() / B.vol[M].sum(), prob.nu)
        assert np.isclose(beta, 9.0 / (32.0 * (lam + 4 * G)), rtol=1e-14)
    # macro-wise constants span the kernel
    macro_id = np.zeros(prob.n_cells, int)
    for i, M in enumerate(B.macro):
        macro_id[M] = i
    v = np.random.default_rng(0).standard_normal(B.macro.shape[0])[macro_id]
    assert np.abs(A @ v).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.matrix_rank(A) == prob.n_cells - B.macro.shape[0]


def test_stabilization_pattern_inside_ppi_pip_pattern():
    B = assemble_blocks(_small(4))
    P = (abs(B.A_ppi) @ abs(B.A_pip)).tocsr()
    S = abs(B.A_stab).tocsr()
    S.eliminate_zeros()
    assert ((S != 0).astype(int) - (S != 0).multiply(P != 0).astype(int)).nnz == 0


def test_condensed_element_zero_flux_identity():
    B = assemble_blocks(make_config("perturbed96", n=4))
    # pi = p on every face of a cell => no flux: rows [dt alpha, -dt g^T] and [-g, M^-1] annihilate 1
    assert np.allclose(B.dt * B.alpha - B.dt * B.g.sum(axis=1), 0, atol=1e-15 * B.alpha.max())
    assert np.allclose(-B.g + B.Minv.sum(axis=2), 0, atol=1e-15 * np.abs(B.g).max())
    assert np.all(B.alpha > 0)


@pytest.mark.parametrize("name", ["unit8", "perturbed96"])
def test_local_mass_conservation(name):
    prob = make_config(name, n=4)
    r = solve_step(prob)
    B = r["B"]
    res = mass_residual(B, r["u"], r["p"], r["pi"], include_stab=True)
    # the balance sums the volumetric, flux and stabilization terms; its
    # rounding is relative to the largest of them (the face fluxes here)
    scale = max(np.abs(B.A_pu @ r["u"]).max(), B.dt * np.abs(r["w"]).max(), np.abs(B.A_stab @ r["p"]).max())
    assert np.abs(res).max() < 1e-10 * scale
    # without the fictitious stabilization flux: conserved per macro-element only
    res0 = mass_residual(B, r["u"], r["p"], r["pi"], include_stab=False)
    assert np.abs(res0).max() > 1e-3 * scale
    assert np.abs(res0[B.macro].sum(axis=1)).max() < 1e-10 * scale
    # flux continuity on interior faces, zero flux on no-flow faces
    w = r["w"]
    F = B.mesh.cell_faces
    tot = np.zeros(B.n_pi)
    np.add.at(tot, F.ravel(), w.ravel())
    free = ~B.pi_fixed
    assert np.abs(tot[free]).max() < 1e-10 * np.abs(w).max()


def test_stabilization_conserves_with_storage_per_cell_when_off():
    prob = make_config("cube64", n=4, S_eps=1e-4).with_(stabilize=False)
    r = solve_step(prob)
    res = mass_residual(r["B"], r["u"], r["p"], r["pi"], include_stab=False)
    B = r["B"]
    scale = max(np.abs(B.A_pu @ r["u"]).max(), B.dt * np.abs(r["w"]).max())
    assert np.abs(res).max() < 1e-10 * scale


def test_spurious_pressure_modes_removed_by_stabilization():
    n = 4
    prob = _small(n)
    B = assemble_blocks(prob)
    m = B.mesh
    i, j, k = m.node_ijk()
    bd = (i == 0) | (i == n) | (j == 0) | (j == n) | (k == 0) | (k == n)
    free = np.repeat(~bd, 3)
    Auu = B.A_uu.toarray()[np.ix_(free, free)]
    Aup = B.A_up.toarray()[free]
    S = Aup.T @ np.linalg.solve(Auu, Aup)           # undrained Schur complement
    ev = np.linalg.eigvalsh(S)
    nker = int((ev < 1e-10 * ev.max()).sum())
    assert nker > 1                                   # constants plus spurious modes
    cb = (-1.0) ** (m.ci + m.cj + m.ck)
    assert np.linalg.norm(S @ cb) < 1e-12 * ev.max() * np.linalg.norm(cb)
    St = S + B.A_stab.toarray()
    ev2 = np.linalg.eigvalsh(St)
    assert int((ev2 < 1e-10 * ev2.max()).sum()) == 1   # only the constant pressure
    assert cb @ St @ cb > 1e-3 * ev2.max() * (cb @ cb)


def test_stabilization_reduces_checkerboard_undrained():
    base = make_config("unit8", n=8).with_(dt=1e-8)
    p_s = solve_step(base)["p"]
    p_n = solve_step(base.with_(stabilize=False))["p"]
    m = solve_step(base)["B"].mesh
    cb = (-1.0) ** (m.ci + m.cj + m.ck)
    assert abs(cb @ p_s) < 0.2 * abs(cb @ p_n)


def test_terzaghi_first_order_convergence():
    errs = []
    T = 0.01
    for nz, ns in [(8, 4), (16, 8), (32, 16)]:
        nc = 4 * nz
        prob = Problem("terz", 2, 2, nz, uniform_coords(2, 2, nz), np.full(nc, 1e4),
                       np.full((nc, 3), 1e-3), nu=0.25, S_eps=0.0, dt=T / ns, rollers=True)
        u = p = None
        for _ in range(ns):
            A, b, B = build_system(prob, None, u, p)
            u, p, pi = split(B, direct_solve(A, b))
        lam, G = lame(1e4, 0.25)
        cv = terzaghi.consolidation_coefficient(1e-3, 1.0, 0.0, 1.0, lam, G)
        assert np.isclose(cv, 12.0)
        p0 = terzaghi.initial_pressure(1.0, 0.0, 1.0, lam, G)
        zc = (np.arange(nz) + 0.5) / nz
        pex = terzaghi.pressure(1.0 - zc, T, 1.0, cv, p0)
        pc = p.reshape(nz, 4)
        assert np.abs(pc - pc[:, :1]).max() < 1e-9          # one-dimensional
        errs.append(np.linalg.norm(pc[:, 0] - pex) / np.linalg.norm(pex))
    assert errs[0] < 0.05
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.9) and np.all(rates < 1.2)


def test_terzaghi_series_initial_condition():
    z = np.linspace(0.05, 1.0, 12)
    assert np.allclose(terzaghi.pressure(z, 0.0, 1.0, 12.0, 1.0, terms=20000), 1.0, atol=2e-3)


def _tiny_system(n=2, dt=1e-2, stabilize=True):
    prob = _small(n, dt=dt).with_(stabilize=stabilize)
    A, b, B = build_system(prob)
    return prob, A, b, B


def test_theorem1_and_lemma1_spectrum():
    prob, A, b, B = _tiny_system(2)
    P = BlockPrec(B)
    N = A.shape[0]
    Minv = np.column_stack([P.apply(e) for e in np.eye(N)])
    T = A.toarray() @ Minv
    ev = np.linalg.eigvals(T)
    n_u = int((~B.u_fixed).sum())
    n_pi = int((~B.pi_fixed).sum())
    n_p = B.n_p
    ones = int((np.abs(ev - 1.0) < 1e-8).sum())
    assert ones >= n_u + n_pi - n_p
    # Lemma 1 (2-norms on the free p/pi blocks)
    Auu, Aup, Apu, Appi, Apip, Apipi = masked_blocks(B)
    Auu_d = Auu.toarray()
    Bp = (B.App_bar + B.A_stab).toarray() - Apu.toarray() @ np.linalg.solve(Auu_d, Aup.toarray())
    Bt = np.diag(P.bp)
    Ep = Bp @ np.linalg.inv(Bt) - np.eye(n_p)
    fpi = ~B.pi_fixed
    C = P.C.toarray()[np.ix_(fpi, fpi)]
    Appi_f = Appi.toarray()[:, fpi]
    Apip_f = Apip.toarray()[fpi]
    Z = np.block([[Ep, -B.dt * Ep @ Appi_f @ np.linalg.inv(C)],
                  [Apip_f @ np.linalg.inv(Bt), np.zeros((fpi.sum(), fpi.sum()))]])
    mu = np.linalg.eigvals(Z)
    eps = np.linalg.norm(Ep, 2) / 2
    gam = np.linalg.norm(Appi_f @ np.linalg.inv(C) @ Apip_f @ np.linalg.inv(Bt), 2)
    bound = eps + np.sqrt(eps ** 2 + 2 * B.dt * gam * eps)
    assert np.abs(mu).max() <= bound * (1 + 1e-10)
    # the eigenvalues of T off 1 are 1 + mu for the nonzero mu
    mu_nz = mu[np.abs(mu) > 1e-8]
    for m_ in mu_nz:
        assert np.min(np.abs(ev - (1 + m_))) < 1e-6 * max(1, abs(m_))


def test_theorem2_remark_and_lemma2():
    prob, A, b, B = _tiny_system(2)
    Auu, Aup, Apu, Appi, Apip, Apipi = masked_blocks(B)
    fpi = ~B.pi_fixed
    Bp = (B.App_bar + B.A_stab).toarray() - Apu.toarray() @ np.linalg.solve(Auu.toarray(), Aup.toarray())
    Cpi = Apipi.toarray() - B.dt * Apip.toarray() @ np.linalg.solve(Bp, Appi.toarray())
    Cf = Cpi[np.ix_(fpi, fpi)]
    assert np.allclose(Cf, Cf.T, rtol=1e-10, atol=1e-14 * np.abs(Cf).max())
    assert np.linalg.eigvalsh(0.5 * (Cf + Cf.T)).min() > 0          # Theorem 2
    Ct = cpi_tilde(B).toarray()[np.ix_(fpi, fpi)]
    assert np.allclose(Ct, Ct.T)
    assert np.linalg.eigvalsh(Ct).min() > 0                          # remark after eq. app_Bp
    # Lemma 2: every eigenvalue decreases with dt and stays above the dt->inf bound
    lams = []
    dts = [1e-6, 1e-4, 1e-2, 1.0, 1e2]
    for dt in dts:
        Bd = assemble_blocks(prob, dt)
        lams.append(np.linalg.eigvalsh(cpi_tilde(Bd).toarray()[np.ix_(fpi, fpi)]))
    lams = np.array(lams)
    assert np.all(np.diff(lams, axis=0) <= 1e-12 * lams.max())
    assert lams.min() > 0
    # Rayleigh-quotient form of Lemma 2 for the eigenvectors at one dt
    Bd = assemble_blocks(prob, 1e-2)
    Ct = cpi_tilde(Bd).toarray()[np.ix_(fpi, fpi)]
    w, V = np.linalg.eigh(Ct)
    App = Apipi.toarray()[np.ix_(fpi, fpi)]
    c = P_c = bp_tilde(Bd) - Bd.dt * Bd.alpha                         # diag(H~)
    d = Bd.alpha
    for idx in [0, len(w) // 2, len(w) - 1]:
        v = V[:, idx]
        bb = Appi.toarray()[:, fpi] @ v
        lam = v @ App @ v - np.sum(bb ** 2 * Bd.dt / (c + d * Bd.dt))
        assert np.isclose(lam, w[idx], rtol=1e-9)


def test_fgmres_block_preconditioner_matches_direct():
    prob = make_config("unit8")
    A, b, B = build_system(prob)
    x = direct_solve(A, b)
    P = BlockPrec(B)
    xg, its, _ = fgmres(lambda v: A @ v, b, P.apply, rtol=1e-14)
    for a, c in zip(split(B, xg), split(B, x)):
        assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(c)
    assert its < 60
    # M^-T is the transpose of M^-1
    N = A.shape[0]
    rng = np.random.default_rng(1)
    x1, y1 = rng.standard_normal(N), rng.standard_normal(N)
    assert np.isclose(y1 @ P.apply(x1), x1 @ P.apply_transpose(y1), rtol=1e-10)


def test_fgmres_unpreconditioned_small_system():
    # GMRES on a tiny nonsymmetric system reaches the direct solution
    rng = np.random.default_rng(3)
    A = sp.csr_matrix(np.eye(30) * 4 + rng.standard_normal((30, 30)) * 0.3)
    b = rng.standard_normal(30)
    x, its, _ = fgmres(lambda v: A @ v, b, None, rtol=1e-13, restart=10)
    assert np.allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-10)


def test_adjoint_matches_central_differences_single_step():
    prob = make_config("perturbed96", n=4)
    r = single_step(prob, prob.obs_cells)
    d = 1e-3
    # the losses carry a rounding error of ~1e-13 of their value (direct
    # solves), which their central difference divides by 2d
    floor = 1e-12 * r["loss"] / d
    for T in prob.fd_cells[:6]:
        kp, km = prob.kappa.copy(), prob.kappa.copy()
        kp[T] *= np.exp(d)
        km[T] *= np.exp(-d)
        fd = (forward_loss(prob.with_(kappa=kp), prob.obs_cells) -
              forward_loss(prob.with_(kappa=km), prob.obs_cells)) / (2 * d)
        assert abs(fd - r["dlogk"][T]) <= 2e-5 * abs(r["dlogk"][T]) + floor
        Ep, Em = prob.E.copy(), prob.E.copy()
        Ep[T] *= np.exp(d)
        Em[T] *= np.exp(-d)
        fd = (forward_loss(prob.with_(E=Ep), prob.obs_cells) -
              forward_loss(prob.with_(E=Em), prob.obs_cells)) / (2 * d)
        assert abs(fd - r["dlogE"][T]) <= 2e-5 * abs(r["dlogE"][T]) + floor


def test_adjoint_matches_central_differences_multi_step():
    prob = make_config("spe192", n=2)
    dts = prob.dts[:4]
    r = multi_step(prob, dts, prob.obs_cells)
    d = 1e-3
    floor = 1e-12 * r["loss"] / d
    for T in [0, 5, 11, 30]:
        kp, km = prob.kappa.copy(), prob.kappa.copy()
        kp[T] *= np.exp(d)
        km[T] *= np.exp(-d)
        fd = (forward_loss(prob.with_(kappa=kp), prob.obs_cells, dts) -
              forward_loss(prob.with_(kappa=km), prob.obs_cells, dts)) / (2 * d)
        assert abs(fd - r["dlogk"][T]) <= 2e-5 * abs(r["dlogk"][T]) + floor
        Ep, Em = prob.E.copy(), prob.E.copy()
        Ep[T] *= np.exp(d)
        Em[T] *= np.exp(-d)
        fd = (forward_loss(prob.with_(E=Ep), prob.obs_cells, dts) -
              forward_loss(prob.with_(E=Em), prob.obs_cells, dts)) / (2 * d)
        assert abs(fd - r["dlogE"][T]) <= 2e-5 * abs(r["dlogE"][T]) + floor


def test_dirichlet_rows_hold_prescribed_values():
    prob = make_config("unit8", n=4).with_(p_top=0.25)
    A, b, B = build_system(prob)
    x = direct_solve(A, b)
    u, p, pi = split(B, x)
    assert np.all(u[B.u_fixed] == 0.0)
    assert np.allclose(pi[B.pi_fixed], 0.25)


def test_sampled_rows_equal_full_assembly():
    from oracle.sampled import system_rows
    for prob in (make_config("perturbed96", n=4), make_config("layered128", n=4).with_(p_top=0.2)):
        A, b, B = build_system(prob)
        rng = np.random.default_rng(5)
        rows = np.unique(np.concatenate([rng.choice(B.n_u, 12, replace=False),
                                         B.n_u + rng.choice(B.n_p, 8, replace=False),
                                         B.n_u + B.n_p + rng.choice(B.n_pi, 12, replace=False),
                                         [0, B.n_u - 1, B.n_u + B.n_p + B.n_pi - 1]]))
        Ar, br = system_rows(prob, rows)
        assert abs(Ar - A[rows]).max() <= 1e-12 * abs(A).max()
        assert np.allclose(br, b[rows], rtol=1e-12, atol=1e-15 * np.abs(b).max())


@pytest.mark.parametrize("dt", [0.1, 1e-5])
def test_cantilever_impermeable_volume_conservation(dt):
    """Cantilever (Sec. 5.2): no face is drained, so summing the p-rows over
    all cells cancels every flux (interior faces by the pi-rows' continuity,
    boundary faces by their zero-flux rows) and the stabilization (rows of
    L_cube sum to zero): from rest, S_eps = 0 leaves sum_T (A_pu u)_T = 0,
    the discrete undrained volume balance.  The drained column problem of the
    same size does not satisfy it (fluid leaves through the top)."""
    from synth import cantilever
    prob = cantilever(4, dt)
    A, b, B = build_system(prob)
    assert not B.pi_fixed.any()
    fixed_nodes = np.nonzero(B.u_fixed.reshape(-1, 3).all(axis=1))[0]
    assert len(fixed_nodes) == 5 * 5  # the face x = 0
    u, p, pi = split(B, direct_solve(A, b))
    vol = B.A_pu @ u
    assert abs(vol.sum()) <= 1e-10 * np.abs(vol).sum()
    col = Problem("c", 4, 4, 4, prob.coords, prob.E, prob.kappa, nu=prob.nu, biot=1.0, S_eps=0.0, mu=prob.mu,
                  dt=dt)
    A2, b2, B2 = build_system(col)
    u2, _, _ = split(B2, direct_solve(A2, b2))
    v2 = B2.A_pu @ u2
    assert abs(v2.sum()) > 1e-3 * np.abs(v2).sum()


def test_cantilever_mirror_symmetry():
    """The homogeneous cantilever is symmetric under the reflection y -> 1 - y:
    u_x, u_z and p are even, u_y is odd (a transposed index or a wrong sign
    in the face coupling breaks it)."""
    from synth import cantilever
    n = 4
    prob = cantilever(n, 1e-2)
    A, b, B = build_system(prob)
    u, p, pi = split(B, direct_solve(A, b))
    U = u.reshape(n + 1, n + 1, n + 1, 3)  # [k, j, i, comp]
    P = p.reshape(n, n, n)
    s = np.abs(U).max()
    assert np.abs(U[:, ::-1, :, 0] - U[..., 0]).max() <= 1e-9 * s
    assert np.abs(U[:, ::-1, :, 2] - U[..., 2]).max() <= 1e-9 * s
    assert np.abs(U[:, ::-1, :, 1] + U[..., 1]).max() <= 1e-9 * s
    assert np.abs(P[:, ::-1, :] - P).max() <= 1e-9 * np.abs(P).max()
