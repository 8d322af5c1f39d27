"""Closed-form pins of the oracle's preconditioner pieces (CPU only).

On a box of identical rectangular cells (edges hx, hy, hz, volume V) with a
uniform Young's modulus and a diagonal permeability per cell, every quantity
the block preconditioners are built from has a closed form that follows from
the Q1 and RT0 bases alone.  The expected values below are written out from
those bases, cell by cell and face by face, without any oracle code:

* Q1 (Appendix A, eq. MFE_matrix): the node function N_a of a cell has
  int_T dN_a/dx_c = +-V/(4 h_c) (divergence theorem: N_a integrates to
  V/(4 h_c) on the one face normal to x_c where it is non-zero), so every
  coupling entry is (A_up)_{(a,c),T} = -+ b V/(4 h_c); and
  int_T (dN_a/dx_d)^2 = V/(9 h_d^2), so the diagonal stiffness of dof (a, c)
  from one cell is (V/9) ((lambda+2G)/h_c^2 + G sum_{d != c} 1/h_d^2).  A
  node shared by m cells has m times that.
* RT0 on a box with diagonal kappa (Sec. 2.2): M_T couples only the two
  faces of each direction, block (mu h_d^2/(kappa_d V)) [[1/3,-1/6],[-1/6,1/3]]
  in the outward unit-flux basis, inverse (kappa_d V/(mu h_d^2)) [[4,2],[2,4]];
  g = M^-1 1 is 6 kappa_d V/(mu h_d^2) on both faces of direction d and
  alpha = sum_d 12 kappa_d V/(mu h_d^2).
* Stabilization (Sec. 3, eq. J_def): beta = (3b)^2/(32(lambda+4G)) with
  |M| = 8V, diagonal 3 beta |M| and -beta |M| between face neighbours of one
  macro-element.

With these, B~_p (eq. app_Bp, the explicit diagonal of variant M_I^(h)),
C~_pi (Sec. 4) and the MFE C~_p of eq. prec (Sec. 5, lumped A_qq) are
checked entry by entry.  A dropped square, the diagonal of a fixed dof in the
fixed-stress sum, a fixed dof counted, a missing dt or a wrong lumping fails
them.  The last tests check the qualitative statement of table tab:can_1
that stabilization removes a degradation of the block preconditioners at
small time steps on the 3D cantilever.
"""
import numpy as np
import pytest

from oracle.mfe import assemble_mfe, build_mfe_system, BtpPrec, cp_tilde, lumped_aqq
from oracle.solve import BlockPrec, bp_tilde, cpi_tilde, fgmres
from oracle.system import assemble_blocks, build_system
from synth import Problem, cantilever, uniform_coords

NX, NY, NZ = 4, 6, 4
L = (1.0, 0.9, 0.5)
E0, NU, BIOT, MU = 3e4, 0.3, 0.8, 2.0


def _lame():
    lam = E0 * NU / ((1 + NU) * (1 - 2 * NU))
    return lam, E0 / (2 * (1 + NU))


def _box(kind, S_eps=1e-4, dt=0.05, seed=4):
    nc = NX * NY * NZ
    rng = np.random.default_rng(seed)
    kappa = 1e-3 * np.exp(rng.standard_normal((nc, 3)))
    return Problem("box", NX, NY, NZ, uniform_coords(NX, NY, NZ, *L), np.full(nc, E0), kappa, nu=NU,
                   biot=BIOT, S_eps=S_eps, mu=MU, dt=dt, rollers=(kind == "rollers"),
                   bc="cantilever" if kind == "cantilever" else "column")


def _h():
    return np.array([L[0] / NX, L[1] / NY, L[2] / NZ])


def _cell(i, j, k):
    return i + NX * (j + NY * k)


def _face(d, i, j, k):
    """Face of direction d whose lower corner is node (i, j, k), in the
    numbering of the C header: x-normal, then y-normal, then z-normal."""
    nfx = (NX + 1) * NY * NZ
    nfy = NX * (NY + 1) * NZ
    if d == 0:
        return i + (NX + 1) * (j + NY * k)
    if d == 1:
        return nfx + i + NX * (j + (NY + 1) * k)
    return nfx + nfy + i + NX * (j + NY * k)


def _cells():
    for k in range(NZ):
        for j in range(NY):
            for i in range(NX):
                yield i, j, k


def _cell_faces(i, j, k):
    """(direction, face below, face above) per direction."""
    return [(0, _face(0, i, j, k), _face(0, i + 1, j, k)), (1, _face(1, i, j, k), _face(1, i, j + 1, k)),
            (2, _face(2, i, j, k), _face(2, i, j, k + 1))]


def _node_fixed(kind, ni, nj, nk, c):
    if kind == "cantilever":
        return ni == 0
    if nk == 0:
        return True
    if kind == "rollers":
        return (c == 0 and ni in (0, NX)) or (c == 1 and nj in (0, NY))
    return False


def _drained_faces(kind):
    if kind == "cantilever":
        return set()
    return {_face(2, i, j, NZ) for i in range(NX) for j in range(NY)}


def _fixed_stress(kind):
    """sum over the free dofs of T of (A_up)^2 / (A_uu)_ii."""
    h, V = _h(), float(np.prod(_h()))
    lam, G = _lame()
    out = np.zeros(NX * NY * NZ)
    for (i, j, k) in _cells():
        s = 0.0
        for a in range(8):
            ni, nj, nk = i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1)
            m = 1
            for v, n in ((ni, NX), (nj, NY), (nk, NZ)):
                m *= 1 if v in (0, n) else 2
            for c in range(3):
                if _node_fixed(kind, ni, nj, nk, c):
                    continue
                aup2 = (BIOT * V / (4 * h[c])) ** 2
                kdiag = m * V / 9.0 * ((lam + 2 * G) / h[c] ** 2 + G * sum(1 / h[d] ** 2 for d in range(3) if d != c))
                s += aup2 / kdiag
        out[_cell(i, j, k)] = s
    return out


def _beta_M():
    lam, G = _lame()
    return (3 * BIOT) ** 2 / (32 * (lam + 4 * G)) * 8 * float(np.prod(_h()))


def _bp_closed(prob, kind):
    h, V = _h(), float(np.prod(_h()))
    alpha = (12 * prob.kappa * V / (prob.mu * h[None, :] ** 2)).sum(axis=1)
    return prob.S_eps * V + prob.dt * alpha + 3 * _beta_M() + _fixed_stress(kind)


@pytest.mark.parametrize("kind", ["column", "rollers", "cantilever"])
def test_bp_tilde_closed_form(kind):
    prob = _box(kind)
    B = assemble_blocks(prob)
    want = _bp_closed(prob, kind)
    got = bp_tilde(B)
    assert np.abs(got - want).max() <= 1e-12 * want.max()
    # the fixed-stress term of a cell whose eight nodes are interior is 6 beta_M |T| on cubes
    lam, G = _lame()
    beta = (3 * BIOT) ** 2 / (32 * (lam + 4 * G))
    cube = Problem("cube", 4, 4, 4, uniform_coords(4, 4, 4), np.full(64, E0), np.full((64, 3), 1e-3), nu=NU,
                   biot=BIOT, S_eps=0.0, mu=MU, dt=0.05)
    Bc = assemble_blocks(cube)
    fs = bp_tilde(Bc) - cube.dt * Bc.alpha - 3 * beta * 8 * Bc.vol
    inner = 1 + 4 * (1 + 4 * 1)  # cell (1, 1, 1): all eight nodes interior
    assert np.isclose(fs[inner], 6 * beta * Bc.vol[inner], rtol=1e-12)
    assert np.isclose(fs[inner], 27 * BIOT ** 2 * Bc.vol[inner] / (16 * (lam + 4 * G)), rtol=1e-12)


@pytest.mark.parametrize("kind", ["column", "cantilever"])
def test_cpi_tilde_closed_form(kind):
    prob = _box(kind)
    B = assemble_blocks(prob)
    h, V = _h(), float(np.prod(_h()))
    bp = _bp_closed(prob, kind)
    nf = B.n_pi
    C = np.zeros((nf, nf))
    for (i, j, k) in _cells():
        T = _cell(i, j, k)
        faces, gvals = [], []
        for d, f0, f1 in _cell_faces(i, j, k):
            m = prob.kappa[T, d] * V / (prob.mu * h[d] ** 2)
            blk = m * np.array([[4.0, 2.0], [2.0, 4.0]])
            for r, fr in enumerate((f0, f1)):
                for s, fs in enumerate((f0, f1)):
                    C[fr, fs] += blk[r, s]
            faces += [f0, f1]
            gvals += [6 * m, 6 * m]
        g = np.array(gvals)
        C[np.ix_(faces, faces)] -= prob.dt / bp[T] * np.outer(g, g)
    for f in _drained_faces(kind):
        C[f, :] = 0.0
        C[:, f] = 0.0
        C[f, f] = 1.0
    got = cpi_tilde(B).toarray()
    assert np.abs(got - C).max() <= 1e-12 * np.abs(C).max()


@pytest.mark.parametrize("kind", ["column", "cantilever"])
def test_mfe_lumped_aqq_and_cp_tilde_closed_form(kind):
    prob = _box(kind)
    K = assemble_mfe(prob)
    h, V = _h(), float(np.prod(_h()))
    nf, nc = K.n_q, NX * NY * NZ
    drained = _drained_faces(kind)
    ncell = np.zeros(nf, int)
    for (i, j, k) in _cells():
        for d, f0, f1 in _cell_faces(i, j, k):
            ncell[f0] += 1
            ncell[f1] += 1
    fixed = np.array([ncell[f] == 1 and f not in drained for f in range(nf)])
    # absolute row sums of the masked, oriented A_qq
    Lq = np.where(fixed, 1.0, 0.0)
    for (i, j, k) in _cells():
        T = _cell(i, j, k)
        for d, f0, f1 in _cell_faces(i, j, k):
            c = prob.mu * h[d] ** 2 / (prob.kappa[T, d] * V)
            for f, other in ((f0, f1), (f1, f0)):
                if fixed[f]:
                    continue
                Lq[f] += c / 3.0 + (0.0 if fixed[other] else c / 6.0)
    assert np.abs(lumped_aqq(K) - Lq).max() <= 1e-12 * Lq.max()
    # C~_p = A_stab + S|T| + fixed stress + dt A_qp^T L^-1 A_qp, A_qp[e, T] = -s_{T,e}
    C = np.diag(prob.S_eps * V + _fixed_stress(kind))
    bM = _beta_M()
    for (i, j, k) in _cells():
        T = _cell(i, j, k)
        for d, f0, f1 in _cell_faces(i, j, k):
            for f, sgn in ((f0, -1.0), (f1, 1.0)):
                if fixed[f]:
                    continue
                C[T, T] += prob.dt / Lq[f]
                nb = [i, j, k]
                nb[d] += int(sgn)
                if 0 <= nb[0] < NX and 0 <= nb[1] < NY and 0 <= nb[2] < NZ:
                    C[T, _cell(*nb)] -= prob.dt / Lq[f]
            # stabilization: face neighbour inside the same 2x2x2 macro-element
            nb = [i, j, k]
            nb[d] ^= 1
            C[T, T] += bM
            C[T, _cell(*nb)] -= bM
    got = cp_tilde(K).toarray()
    assert np.abs(got - C).max() <= 1e-12 * np.abs(C).max()


def _its(A, b, P, rtol=1e-6):
    return fgmres(lambda v: A @ v, b, P.apply, rtol=rtol, restart=1000, max_it=400)[1]


def test_tab_can1_mfe_stabilization_removes_small_dt_degradation():
    """tab:can_1, M_I^(m): at dt = 1e-5 the unstabilized MFE system needs far
    more iterations than the stabilized one; at dt = 0.1 the two coincide.
    The right-hand side is a seeded random vector: the unit top load alone,
    on the unscaled system, leaves pressure-block residuals below 1e-6 of
    ||b|| after the displacement solve, so it cannot show the difference."""
    n = 6
    res = {}
    for dt in (0.1, 1e-5):
        for stab in (False, True):
            A, b, K = build_mfe_system(cantilever(n, dt, stabilize=stab))
            r = np.random.default_rng(0).standard_normal(b.size)
            res[dt, stab] = _its(A, r, BtpPrec(K))
    assert res[1e-5, False] >= 1.4 * res[1e-5, True], res
    assert abs(res[0.1, False] - res[0.1, True]) <= 1, res


def test_tab_can1_hybrid_stabilization_clusters_spectrum():
    """tab:can_1, M_I^(h) at dt = 1e-5 on the 4^3 cantilever: stabilization
    moves most eigenvalues of A_H M^-1 that lie far from 1 (Theorem 1: the
    others equal 1) towards it.  The extreme ones stay, which is why the
    oracle's iteration counts do not show the table's jump (see the design
    notes)."""
    far = {}
    for stab in (False, True):
        A, b, B = build_system(cantilever(4, 1e-5, stabilize=stab))
        P = BlockPrec(B)
        N = A.shape[0]
        Mi = np.column_stack([P.apply(e) for e in np.eye(N)])
        ev = np.linalg.eigvals(A.toarray() @ Mi)
        far[stab] = int(np.sum(np.abs(ev - 1) > 0.5))
        assert np.sum(np.abs(ev - 1) > 1e-8) <= 2 * B.n_p
    assert far[True] * 2 <= far[False], far
