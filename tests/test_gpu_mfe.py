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
    for _ in range(6):
        r = b - C @ x
        x = x + s.apply(_capi.PM_OP_VCYCLE_CP, torch.as_tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(b - C @ x) < 0.05 * np.linalg.norm(b)
