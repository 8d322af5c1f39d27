"""Full-size checks in the launch configurations the benchmark times.

The oracle cannot factor these systems.  At 64^3 (both storage values) and
at the perturbed 96^3 mesh it assembles the whole FP64 system A_H, b and
evaluates the full residual of the GPU solution, the GPU operator applied to
it and the per-cell mass balance.  At 128^3 it assembles sampled rows of A_H
and b one by one from the element integrals of their support cells
(``oracle.sampled``): the GPU right-hand side and the GPU operator applied to
the GPU solution agree with the oracle's rows entrywise (FP64, 1e-12 of the
row scale), and the sampled residual entries of the GPU solution are within
the solver tolerance of ||b||."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.sampled import system_rows  # noqa: E402
from oracle.solve import mass_residual, reconstruct_w  # noqa: E402
from oracle.system import build_system, split  # noqa: E402
from paper_2002_09603_amd import _capi  # noqa: E402
from paper_2002_09603_amd.solver import Options, from_problem  # noqa: E402
from synth import make_config  # noqa: E402

BENCH_OPTS = dict(rtol=1e-8, precond_fp32=True, restart=24, max_it=1000, orth_passes=1, cheb_degree_pi=1,
                  cheb_lower_pi=0.1)

CASES = [
    ("layered128", None, 0.0, BENCH_OPTS),
    ("cube64", None, 0.0, dict(rtol=1e-8, restart=50)),
    ("cube64", None, 1e-4, dict(rtol=1e-8, restart=50)),
    ("perturbed96", None, 0.0, dict(rtol=1e-8, restart=50)),
]


@pytest.mark.parametrize("name,n,S,opts", CASES, ids=[f"{c[0]}-S{c[2]}" for c in CASES])
def test_sampled_rows_and_residual_at_full_size(name, n, S, opts):
    prob = make_config(name, n=n, S_eps=S)
    print(f"[full size] {name} {prob.nx}x{prob.ny}x{prob.nz} S_eps={S} N={prob.n_total}", flush=True)
    s = from_problem(prob, Options(**opts)).assemble()
    b = s.build_rhs()
    u, pi, p, info = s.solve(b)
    print("   info", {k: info[k] for k in ("iters", "relres_true", "t_setup", "t_solve")}, flush=True)
    assert info["converged"] and info["relres_true"] <= opts["rtol"]
    x = torch.cat([u, p, pi])
    Ax = s.apply(_capi.PM_OP_AH, x)
    rng = np.random.default_rng(2024)
    n_u, n_p, n_pi = s.n_u, s.n_p, s.n_pi
    rows = np.unique(np.concatenate([
        rng.choice(n_u, 120, replace=False), n_u + rng.choice(n_p, 60, replace=False),
        n_u + n_p + rng.choice(n_pi, 120, replace=False),
        [0, n_u - 1, n_u, n_u + n_p - 1, n_u + n_p, s.N - 1],
        # top-layer nodes (traction) and top faces (drained)
        3 * (prob.n_nodes - 1 - rng.choice((prob.nx + 1) * (prob.ny + 1), 10, replace=False)),
        s.N - 1 - rng.choice(prob.nx * prob.ny, 10, replace=False)]))
    Ar, br = system_rows(prob, rows)
    xh = x.cpu().numpy()
    bh = b.cpu().numpy()
    scale_b = np.abs(Ar) @ np.abs(xh) + np.abs(br) + 1e-300
    assert np.all(np.abs(bh[rows] - br) <= 1e-12 * np.maximum(np.abs(br), np.abs(bh).max() * 1e-3) + 1e-300)
    assert np.all(np.abs(Ar @ xh - Ax.cpu().numpy()[rows]) <= 1e-12 * scale_b)
    res = br - Ar @ xh
    assert np.abs(res).max() <= 1.5 * opts["rtol"] * np.linalg.norm(bh)
    s.close()


def test_mixed_precision_matches_fp64_preconditioner_at_128():
    """The layered 128^3 step with the benchmark's options: the FP32
    preconditioner inside FP64 FGMRES reaches the fields of the FP64
    preconditioner's solve of the same system to 1e-8 relative (L2) per field
    (both to relative residual 1e-8)."""
    prob = make_config("layered128")
    print(f"[mixed vs fp64] layered128 N={prob.n_total}", flush=True)
    fields = {}
    for fp32 in (True, False):
        s = from_problem(prob, Options(**dict(BENCH_OPTS, precond_fp32=fp32))).assemble()
        u, pi, p, info = s.solve(s.build_rhs())
        print("   fp32" if fp32 else "   fp64", {k: info[k] for k in ("iters", "relres_true")}, flush=True)
        assert info["converged"] and info["relres_true"] <= BENCH_OPTS["rtol"]
        fields[fp32] = [f.cpu().numpy() for f in (u, p, pi)]
        s.close()
    for a, b in zip(fields[True], fields[False]):
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)


FULL_CASES = [("cube64", 0.0), ("cube64", 1e-4), ("perturbed96", 0.0)]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,S", FULL_CASES, ids=[f"{c[0]}-S{c[1]}" for c in FULL_CASES])
def test_full_residual_against_oracle_assembly(name, S):
    """The FP64 GPU solve (plain method: FP64 AMG in the block triangular
    preconditioner) of the 64^3 workload with S_eps in {0, 1e-4} and of the
    perturbed 96^3 workload, against the oracle's own assembly of the whole
    system (eq. stab_A with the Dirichlet identity rows): right-hand side
    entrywise, A_H applied to the GPU solution entrywise, the full residual
    ||b - A x|| / ||b|| of the GPU solution at most twice the solver's
    tolerance, and the mass balance of every cell (Sec. 3)."""
    prob = make_config(name, S_eps=S)
    print(f"[full residual] {name} {prob.nx}x{prob.ny}x{prob.nz} S_eps={S} N={prob.n_total}: oracle assembly",
          flush=True)
    A, b, B = build_system(prob)
    print(f"   oracle A_H: {A.nnz} entries", flush=True)
    rtol = 1e-11
    s = from_problem(prob, Options(rtol=rtol, restart=50, max_it=3000)).assemble()
    bg = s.build_rhs().cpu().numpy()
    assert np.abs(bg - b).max() <= 1e-12 * np.abs(b).max()
    u, pi, p, info = s.solve(torch.as_tensor(b, device="cuda"))
    print("   info", {k: info[k] for k in ("iters", "relres_true", "t_setup", "t_solve")}, flush=True)
    assert info["converged"]
    x = torch.cat([u, p, pi])
    xh = x.cpu().numpy()
    Ax = A @ xh
    scale = abs(A) @ np.abs(xh)
    assert np.all(np.abs(s.apply(_capi.PM_OP_AH, x).cpu().numpy() - Ax) <= 1e-12 * scale + 1e-300)
    relres = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    print(f"   oracle residual of the GPU solution {relres:.3e}", flush=True)
    assert relres <= 2 * rtol
    uh, ph, pih = split(B, xh)
    res = mass_residual(B, uh, ph, pih)
    w = reconstruct_w(B, ph, pih)
    bal = max(np.abs(B.A_pu @ uh).max(), B.dt * np.abs(w).max())
    assert np.abs(res).max() <= 1e-8 * bal
    s.close()


def test_perturbed96_adjoint_matches_central_differences_at_full_size():
    """96^3 perturbed mesh, loss = sum of squared pressure at 64 observation
    cells: per-cell d/dlog kappa and d/dlog E from the adjoint against central
    differences (step 1e-3 in log space) on the workload's 16 cells.

    At this size one cell changes the loss by ~1e-9 of its value, below what
    two independent forward solves resolve, so each perturbed solve starts
    from the unperturbed solution x0: it solves A(theta') dx = b - A(theta') x0
    (relative residual 1e-10 of that small right-hand side) and the loss
    difference is summed as (dp+ - dp-)(2 p0 + dp+ + dp-) without
    cancellation.  The perturbed states are still exact solutions of the
    perturbed systems, so this is the plain central difference."""
    from paper_2002_09603_amd.autograd import poro_step

    prob = make_config("perturbed96")
    print(f"[full-size finite differences] perturbed {prob.nx}^3 N={prob.n_total}", flush=True)
    assert np.allclose(prob.kappa, prob.kappa[:, :1])
    s = from_problem(prob, Options(rtol=1e-12, rtol_transpose=1e-10, restart=50, max_it=3000))
    logk = torch.tensor(np.log(prob.kappa[:, 0]), dtype=torch.float64, device="cuda", requires_grad=True)
    logE = torch.tensor(np.log(prob.E), dtype=torch.float64, device="cuda", requires_grad=True)
    obs = torch.as_tensor(prob.obs_cells, device="cuda")
    u, pi, p = poro_step(s, logk, logE)
    (p[obs] ** 2).sum().backward()
    x0 = torch.cat([u, p, pi]).detach()
    p0 = p.detach()[obs]
    d = 1e-3
    worst = 0.0
    for T in prob.fd_cells:
        for which in ("k", "E"):
            dps = []
            for sign in (1.0, -1.0):
                lk, lE = logk.detach().clone(), logE.detach().clone()
                (lk if which == "k" else lE)[int(T)] += sign * d
                kappa = torch.exp(lk)[:, None].expand(-1, 3).contiguous()
                s.update_material(torch.exp(lE).contiguous(), kappa)
                r = s.build_rhs() - s.apply(_capi.PM_OP_AH, x0)
                du, dpi, dp, info = s.solve(r)
                dps.append(dp[obs])
            fd = float(((dps[0] - dps[1]) * (2 * p0 + dps[0] + dps[1])).sum()) / (2 * d)
            ad = float((logk.grad if which == "k" else logE.grad)[int(T)])
            err = abs(fd - ad) / max(abs(ad), 1e-300)
            worst = max(worst, err)
            print(f"   cell {int(T)} d/dlog{which}: adjoint {ad:.10e} fd {fd:.10e} rel {err:.1e}", flush=True)
            assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-300
    print(f"   worst relative difference {worst:.2e}", flush=True)
    s.close()


def test_lattice_operator_matches_assembled_matrix_at_64():
    """64^3 cube (sigma 2 permeability, nu 0.3): the matrix-free finest A_uu
    level against the assembled one, in the FP64 operator (1e-13), its
    transpose, and the solved fields (rtol 1e-11, 1e-8 relative per field)."""
    prob = make_config("cube64")
    print("[lattice vs assembled] cube64", flush=True)
    out = {}
    for lattice in (True, False):
        s = from_problem(prob, Options(rtol=1e-11, restart=50, lattice_uu=lattice)).assemble()
        assert s.info()["lattice_uu"] == int(lattice)
        assert s.info()["lattice_form"] == (3 if lattice else 0)  # cubic cells: the 12-value form
        g = torch.Generator(device="cpu").manual_seed(5)
        x = torch.randn(s.N, generator=g, dtype=torch.float64).cuda()
        y = s.apply(_capi.PM_OP_AH, x)
        yt = s.apply(_capi.PM_OP_AHT, x)
        u, pi, p, info = s.solve(s.build_rhs())
        print(f"   lattice={lattice}: {info['iters']} its, setup {info['t_setup']:.3f} s, "
              f"solve {info['t_solve']:.3f} s", flush=True)
        out[lattice] = (y, yt, u, pi, p)
        s.close()
    a, b = out[True], out[False]
    assert float(torch.linalg.norm(a[0] - b[0]) / torch.linalg.norm(b[0])) <= 1e-13
    assert float(torch.linalg.norm(a[1] - b[1]) / torch.linalg.norm(b[1])) <= 1e-13
    for fa, fb in zip(a[2:], b[2:]):
        assert float(torch.linalg.norm(fa - fb) / torch.linalg.norm(fb)) <= 1e-8
