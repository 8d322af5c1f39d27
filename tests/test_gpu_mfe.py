"""HIP operator of the non-hybridized mixed system (MFE, eq. mfeSys with the
stabilized pressure block) against the oracle's assembled A_M, row block by
row block, and the assembled C~_p of its block triangular preconditioner
(Sec. 5) against the oracle's, through the C ABI.  FP64 on both sides, only
the summation order differs: 1e-12 relative per block.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.mfe import build_mfe_system, cp_tilde, split_mfe  # noqa: E402
from oracle.solve import cpi_tilde  # noqa: E402
from paper_2002_09603_amd import _capi  # noqa: E402
from paper_2002_09603_amd.solver import Options, from_problem  # noqa: E402

from gpu_helpers import box_problem, rel  # noqa: E402

CASES = {
    "box10x6x4": dict(nx=10, ny=6, nz=4, seed=1),
    "perturbed6x8x6": dict(nx=6, ny=8, nz=6, seed=2, perturb=True),
    "rollers4x4x8_ptop": dict(nx=4, ny=4, nz=8, seed=3, rollers=True, p_top=0.3, S_eps=1e-4),
    "cantilever8x6x4": dict(nx=8, ny=6, nz=4, seed=5, bc="cantilever"),
    "cantilever_perturbed6x6x4": dict(nx=6, ny=6, nz=4, seed=6, bc="cantilever", perturb=True, dt=1e-5),
    "unstabilized6x4x4": dict(nx=6, ny=4, nz=4, seed=9, stabilize=False),
    "tiny2x2x2": dict(nx=2, ny=2, nz=2, seed=8),
}


@pytest.mark.parametrize("lattice", [True, False])
@pytest.mark.parametrize("name", list(CASES))
def test_mfe_operator_parity(name, lattice):
    prob = box_problem(**CASES[name])
    print(f"[mfe operator parity] {name} lattice={lattice}", flush=True)
    A, b, K = build_mfe_system(prob)
    s = from_problem(prob, Options(lattice_uu=lattice, stabilize=prob.stabilize)).assemble()
    assert s.N == A.shape[0] and s.n_pi == K.n_q
    rng = np.random.default_rng(11)
    for rep in range(2):                       # the second call reuses the stored cell masses
        x = rng.standard_normal(s.N)
        y = s.apply(_capi.PM_OP_MFE, torch.as_tensor(x, device="cuda")).cpu().numpy()
        ref = A @ x
        for got, want in zip(split_mfe(K, y), split_mfe(K, ref)):
            assert rel(got, want) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_mfe_cp_tilde_parity(name):
    prob = box_problem(**CASES[name])
    print(f"[mfe C~_p parity] {name}", flush=True)
    A, b, K = build_mfe_system(prob)
    s = from_problem(prob, Options(stabilize=prob.stabilize)).assemble()
    C = cp_tilde(K)
    rng = np.random.default_rng(12)
    for rep in range(2):                       # the second call refills the stored pattern
        x = rng.standard_normal(s.n_p)
        y = s.apply(_capi.PM_OP_CP, torch.as_tensor(x, device="cuda")).cpu().numpy()
        assert rel(y, C @ x) < 1e-12


@pytest.mark.parametrize("case", [dict(nx=16, ny=16, nz=8, seed=21, perturb=True),
                                  dict(nx=16, ny=8, nz=8, seed=22, bc="cantilever", dt=1e-5),
                                  dict(nx=16, ny=16, nz=8, seed=23, graded=True, dt=1.0)])
def test_mfe_cp_vcycle_converges(case):
    """The V-cycle for C~_p as a stationary iteration on the oracle's C~_p
    (a property at any size: the hierarchy itself has no oracle)."""
    prob = box_problem(**case)
    print(f"[mfe C~_p V-cycle] {case}", flush=True)
    K = build_mfe_system(prob)[2]
    C = cp_tilde(K)
    s = from_problem(prob, Options()).assemble()
    rng = np.random.default_rng(13)
    b = rng.standard_normal(s.n_p)
    x = np.zeros_like(b)
    res = [np.linalg.norm(b)]
    for _ in range(6):
        r = b - C @ x
        x = x + s.apply(_capi.PM_OP_VCYCLE_CP, torch.as_tensor(r, device="cuda")).cpu().numpy()
        res.append(np.linalg.norm(b - C @ x))
    # one fixed hierarchy (built on the first call): a steady contraction per cycle
    factors = [res[i + 1] / res[i] for i in range(len(res) - 1)]
    # for comparison, the hybrid system's C~_pi V-cycle on the same grid
    Cpi = cpi_tilde(K.B)
    bp = rng.standard_normal(s.n_pi)
    xp = np.zeros_like(bp)
    rpi = [np.linalg.norm(bp)]
    for _ in range(6):
        xp = xp + s.apply(_capi.PM_OP_VCYCLE_PI, torch.as_tensor(bp - Cpi @ xp, device="cuda")).cpu().numpy()
        rpi.append(np.linalg.norm(bp - Cpi @ xp))
    fpi = [rpi[i + 1] / rpi[i] for i in range(len(rpi) - 1)]
    print("   contraction per cycle: C~_p", [round(f, 3) for f in factors], "C~_pi", [round(f, 3) for f in fpi],
          flush=True)
    assert res[-1] < 0.05 * res[0]
    assert max(factors[2:]) < 0.75


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("name", list(CASES))
def test_mfe_rhs_parity(name):
    """[f_u; f_q; f_p] of the MFE step (eq. MFE_vector) from rest and from a
    previous state, against the oracle's lifted right-hand side."""
    prob = box_problem(**CASES[name])
    print(f"[mfe rhs parity] {name}", flush=True)
    A, b, K = build_mfe_system(prob)
    s = from_problem(prob, Options(stabilize=prob.stabilize)).assemble()
    assert rel(s.build_rhs_mfe().cpu().numpy(), b) < 1e-12
    rng = np.random.default_rng(14)
    up, pp = rng.standard_normal(s.n_u) * 1e-3, rng.standard_normal(s.n_p)
    up[K.B.u_fixed] = 0.0
    A2, b2, _ = build_mfe_system(prob, None, up, pp)
    assert rel(s.build_rhs_mfe(_dev(up), _dev(pp)).cpu().numpy(), b2) < 1e-12
    s.close()


@pytest.mark.parametrize("name", ["box10x6x4", "perturbed6x8x6", "cantilever_perturbed6x6x4"])
def test_btp_is_the_block_lower_triangular_preconditioner(name):
    """PM_OP_BTP against eq. prec assembled from its parts: the u block is the
    A_uu V-cycle of x_u, the q block solves A_qq z_q = x_q to the accuracy of
    five Chebyshev-Jacobi sweeps (checked with the oracle's A_qq), and the p
    block is the C~_p V-cycle of x_p - A_pu z_u - dt A_pq z_q (the coupling
    blocks from the oracle)."""
    from oracle.mfe import masked_mfe_blocks
    prob = box_problem(**CASES[name])
    print(f"[btp structure] {name}", flush=True)
    A, b, K = build_mfe_system(prob)
    Auu, Aup, Apu, Aqq, Aqp, Apq = masked_mfe_blocks(K)
    s = from_problem(prob, Options(stabilize=prob.stabilize)).assemble()
    rng = np.random.default_rng(15)
    x = rng.standard_normal(s.N)
    z = s.apply(_capi.PM_OP_BTP, _dev(x)).cpu().numpy()
    xu, xq, xp = split_mfe(K, x)
    zu, zq, zp = split_mfe(K, z)
    zu_ref = s.apply(_capi.PM_OP_VCYCLE_U, _dev(xu)).cpu().numpy()
    assert rel(zu, zu_ref) < 1e-13
    assert np.linalg.norm(xq - Aqq @ zq) <= 0.05 * np.linalg.norm(xq)
    tp = xp - Apu @ zu - K.dt * (Apq @ zq)
    zp_ref = s.apply(_capi.PM_OP_VCYCLE_CP, _dev(tp)).cpu().numpy()
    assert rel(zp, zp_ref) < 1e-10
    s.close()


MFE_SOLVES = [(n, False) for n in CASES] + [("box10x6x4", True), ("cantilever8x6x4", True)]


@pytest.mark.parametrize("name,fp32ctx", MFE_SOLVES, ids=[f"{n}-fp32ctx={f}" for n, f in MFE_SOLVES])
def test_mfe_solve_parity(name, fp32ctx):
    """The MFE step solved on the GPU (FGMRES with the block triangular
    preconditioner, FP64) against the oracle's direct solve of A_M: u, q, p
    within 1e-8 relative per field.  fp32ctx: the context's hierarchies carry
    FP32 copies (the MFE solve still runs its V-cycles on the FP64 levels)."""
    from oracle.mfe import solve_mfe_step
    prob = box_problem(**CASES[name])
    print(f"[mfe solve parity] {name} fp32ctx={fp32ctx}", flush=True)
    ref = solve_mfe_step(prob)
    s = from_problem(prob, Options(rtol=1e-13, restart=60, max_it=2000, stabilize=prob.stabilize,
                                   precond_fp32=fp32ctx)).assemble()
    u, q, p, info = s.solve_mfe(s.build_rhs_mfe())
    print(f"   {info['iters']} its, C~_p levels {info['levels_pi']}", flush=True)
    assert info["converged"] and info["relres_true"] <= 1e-13
    for got, want in ((u, ref["u"]), (q, ref["q"]), (p, ref["p"])):
        assert rel(got.cpu().numpy(), want) <= 1e-8
    # a second solve reuses the hierarchy and gives bitwise the same fields
    u2, q2, p2, info2 = s.solve_mfe(s.build_rhs_mfe())
    assert info2["iters"] == info["iters"]
    assert torch.equal(u, u2) and torch.equal(q, q2) and torch.equal(p, p2)
    s.close()


def test_mfe_solve_after_set_dt_rebuilds_cp():
    """pm_set_dt changes C~_p (dt A_qp^T L^-1 A_qp): the next MFE solve must use
    the new dt's preconditioner and operator and match the oracle at that dt."""
    from oracle.mfe import solve_mfe_step
    prob = box_problem(**CASES["cantilever8x6x4"])
    s = from_problem(prob, Options(rtol=1e-13, restart=60, max_it=2000)).assemble()
    s.solve_mfe(s.build_rhs_mfe())
    s.set_dt(1e-5)
    ref = solve_mfe_step(prob.with_(dt=1e-5))
    C = cp_tilde(build_mfe_system(prob.with_(dt=1e-5))[2])
    xc = np.random.default_rng(16).standard_normal(s.n_p)
    assert rel(s.apply(_capi.PM_OP_CP, _dev(xc)).cpu().numpy(), C @ xc) < 1e-12
    u, q, p, info = s.solve_mfe(s.build_rhs_mfe())
    assert info["converged"]
    for got, want in ((u, ref["u"]), (q, ref["q"]), (p, ref["p"])):
        assert rel(got.cpu().numpy(), want) <= 1e-8
    s.close()
