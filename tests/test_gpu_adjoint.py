"""Adjoint and time-loop paths on the GPU (through the C ABI), checked against
the FP64 CPU oracle's adjoint and against central finite differences of the
GPU forward solve.

Tolerances: gradients from the GPU adjoint vs. the oracle adjoint 1e-7
relative (the transposed solve is converged to 1e-10, the fields to ~1e-11);
central differences (step 1e-3 in log space, forward solves at relative
residual 1e-12) vs. the adjoint 1e-5 relative per cell; checkpointed vs.
stored-state backward passes bitwise equal (deterministic kernels)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.adjoint import multi_step, single_step  # noqa: E402
from paper_2002_09603_amd.autograd import poro_step, time_loop  # noqa: E402
from paper_2002_09603_amd.solver import Options, from_problem  # noqa: E402
from synth import make_config  # noqa: E402

from gpu_helpers import rel  # noqa: E402

DEV = "cuda"


def _logs(prob):
    logk = torch.tensor(np.log(prob.kappa[:, 0]), dtype=torch.float64, device=DEV, requires_grad=True)
    logE = torch.tensor(np.log(prob.E), dtype=torch.float64, device=DEV, requires_grad=True)
    return logk, logE


def test_step_gradients_match_oracle_adjoint():
    prob = make_config("perturbed96", n=6)
    print("[step adjoint] perturbed 6^3", flush=True)
    ref = single_step(prob, prob.obs_cells)
    s = from_problem(prob, Options(rtol=1e-13, rtol_transpose=1e-10))
    logk, logE = _logs(prob)
    u, pi, p = poro_step(s, logk, logE)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    loss = (p[obs] ** 2).sum()
    assert abs(float(loss) - ref["loss"]) <= 1e-9 * ref["loss"]
    loss.backward()
    assert rel(logk.grad.cpu().numpy(), ref["dlogk"]) <= 1e-7
    assert rel(logE.grad.cpu().numpy(), ref["dlogE"]) <= 1e-7
    s.close()


def test_backward_after_other_forward_passes_on_the_same_solver():
    """Backward re-applies its forward pass's material and time step: two
    more forward passes (other fields, another dt) and a set_dt on the same
    solver between forward and backward leave the gradient unchanged."""
    prob = make_config("perturbed96", n=6)
    print("[interleaved forwards] perturbed 6^3", flush=True)
    ref = single_step(prob, prob.obs_cells)
    s = from_problem(prob, Options(rtol=1e-13, rtol_transpose=1e-10))
    logk, logE = _logs(prob)
    u, pi, p = poro_step(s, logk, logE)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    loss = (p[obs] ** 2).sum()
    with torch.no_grad():
        poro_step(s, logk.detach() + 0.7, logE.detach() - 0.2)
    s.set_dt(3 * prob.dt)
    lk2, lE2 = (logk.detach() - 0.4).requires_grad_(), logE.detach().clone().requires_grad_()
    _, _, p2 = poro_step(s, lk2, lE2)
    loss.backward()
    assert rel(logk.grad.cpu().numpy(), ref["dlogk"]) <= 1e-7
    assert rel(logE.grad.cpu().numpy(), ref["dlogE"]) <= 1e-7
    assert s.dt == prob.dt
    s.close()


def _loss_gpu(s, prob, logk, logE, obs):
    with torch.no_grad():
        u, pi, p = poro_step(s, logk, logE)
        return float((p[obs] ** 2).sum())


@pytest.mark.parametrize("n", [6, 16])
def test_step_gradients_match_central_differences(n):
    prob = make_config("perturbed96", n=n)
    print(f"[finite differences] perturbed {n}^3", flush=True)
    s = from_problem(prob, Options(rtol=1e-12, rtol_transpose=1e-10, max_it=2000))
    logk, logE = _logs(prob)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    u, pi, p = poro_step(s, logk, logE)
    (p[obs] ** 2).sum().backward()
    gk, gE = logk.grad.clone(), logE.grad.clone()
    d = 1e-3
    for T in prob.fd_cells[:4]:
        for g, which in ((gk, "k"), (gE, "E")):
            lk, lE = logk.detach().clone(), logE.detach().clone()
            tgt = lk if which == "k" else lE
            tgt[T] += d
            lp = _loss_gpu(s, prob, lk, lE, obs)
            tgt[T] -= 2 * d
            lm = _loss_gpu(s, prob, lk, lE, obs)
            fd = (lp - lm) / (2 * d)
            ad = float(g[T])
            print(f"   cell {T} d/dlog{which}: adjoint {ad:.8e} fd {fd:.8e}", flush=True)
            assert abs(fd - ad) <= 1e-5 * abs(ad) + 1e-14
    s.close()


def test_time_loop_gradients_match_oracle_and_checkpointing_is_exact():
    prob = make_config("spe192", n=2)           # 4 x 4 x 2 cells, E and kappa heterogeneous
    dts = list(prob.dts[:4])
    print("[time loop adjoint] 4x4x2, 4 steps", flush=True)
    ref = multi_step(prob, dts, prob.obs_cells)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    grads = []
    for every in (1, 2):
        s = from_problem(prob, Options(rtol=1e-13, rtol_transpose=1e-10))
        logk, logE = _logs(prob)
        P = time_loop(s, logk, logE, dts, every=every)
        loss = (P[:, obs] ** 2).sum()
        assert abs(float(loss) - ref["loss"]) <= 1e-9 * ref["loss"]
        loss.backward()
        grads.append((logk.grad.clone(), logE.grad.clone()))
        s.close()
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    assert rel(grads[1][0].cpu().numpy(), ref["dlogk"]) <= 1e-7
    assert rel(grads[1][1].cpu().numpy(), ref["dlogE"]) <= 1e-7


def test_twenty_step_mixed_precision_gradients_match_oracle():
    """The 20-step workload recipe (log-normal kappa sigma 3, E sigma 0.5,
    geometric dt 1e-3 -> 1) on 8 x 8 x 4 cells, mixed-precision forward and
    adjoint with checkpoints every 5 steps, against the oracle's 20-step
    adjoint (direct solves, all states kept)."""
    prob = make_config("spe192", n=4)
    dts = list(prob.dts)
    assert len(dts) == 20
    print("[20-step adjoint] 8x8x4, mixed precision, checkpoints every 5", flush=True)
    ref = multi_step(prob, dts, prob.obs_cells)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    s = from_problem(prob, Options(rtol=1e-13, rtol_transpose=1e-10, precond_fp32=True, max_it=2000))
    logk, logE = _logs(prob)
    P = time_loop(s, logk, logE, dts, every=5)
    loss = (P[:, obs] ** 2).sum()
    assert abs(float(loss) - ref["loss"]) <= 1e-9 * ref["loss"]
    loss.backward()
    print(f"   dlogk rel {rel(logk.grad.cpu().numpy(), ref['dlogk']):.2e} "
          f"dlogE rel {rel(logE.grad.cpu().numpy(), ref['dlogE']):.2e}", flush=True)
    assert rel(logk.grad.cpu().numpy(), ref["dlogk"]) <= 1e-7
    assert rel(logE.grad.cpu().numpy(), ref["dlogE"]) <= 1e-7
    s.close()


def test_twenty_step_checkpointing_and_directional_differences():
    """24 x 24 x 12 cells of the same recipe, 20 steps, mixed precision:
    checkpoints every 5 steps give bitwise the gradients of keeping every
    state, and the gradient's projection on a random direction (v_k, v_E)
    matches the central difference of the 20-step loss (step 1e-3, forward
    solves at relative residual 1e-12) to 1e-5."""
    prob = make_config("spe192", n=12)
    dts = list(prob.dts)
    print(f"[20-step adjoint] {prob.nx}x{prob.ny}x{prob.nz}, mixed precision", flush=True)
    obs = torch.as_tensor(prob.obs_cells, device=DEV)
    s = from_problem(prob, Options(rtol=1e-12, rtol_transpose=1e-10, precond_fp32=True, max_it=2000))
    grads = []
    for every in (1, 5):
        logk, logE = _logs(prob)
        P = time_loop(s, logk, logE, dts, every=every)
        (P[:, obs] ** 2).sum().backward()
        grads.append((logk.grad.clone(), logE.grad.clone()))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    gk, gE = grads[1]
    g = torch.Generator(device="cpu").manual_seed(7)
    vk = torch.randn(prob.n_cells, generator=g, dtype=torch.float64).to(DEV)
    vE = torch.randn(prob.n_cells, generator=g, dtype=torch.float64).to(DEV)
    logk, logE = _logs(prob)
    d = 1e-3
    with torch.no_grad():
        Lp = float((time_loop(s, logk + d * vk, logE + d * vE, dts)[:, obs] ** 2).sum())
        Lm = float((time_loop(s, logk - d * vk, logE - d * vE, dts)[:, obs] ** 2).sum())
    fd = (Lp - Lm) / (2 * d)
    ad = float((gk * vk).sum() + (gE * vE).sum())
    print(f"   directional derivative: adjoint {ad:.10e} fd {fd:.10e}", flush=True)
    assert abs(fd - ad) <= 1e-5 * abs(ad)
    s.close()
