#!/usr/bin/env python3
"""Benchmark of one backward-Euler step of hybridized poromechanics on one GPU.

Workload (default ``layered128``): 128^3 hexahedral unit cube, 14,877,827
unknowns (6,440,067 displacement, 6,340,608 face pressure, 2,097,152 cell
pressure), layered anisotropic permeability (kxx = kyy = 1e-2, kzz = 1e-6 in
alternating 8-cell layers, isotropic 1e-6 in the others, log-normal sigma=1
noise), E = 1e4, nu = 0.25, b = 1, S_eps = 0, dt = 1e-2, bottom fixed, top
loaded and drained.  Mixed precision: AMG V-cycles and the Schur-complement
apply in FP32 inside FP64 flexible GMRES (FP64 residual, Arnoldi, coarse
solves), stopped at a relative residual of 1e-8.

One step = the whole hot path on inputs already resident on the device:
element kernels and static condensation, stabilization, assembly, B~_p,
C~_pi, both AMG setups, right-hand side, the preconditioned FGMRES solve and
the flux reconstruction.  The metric is the step's time to solution (s).

Also reported: iterations and phase times; the roofline of the dominant
operator / V-cycle kernel (algorithmic bytes, or stencil flops for the
matrix-free lattice kernels, over HIP-event durations of its launches inside
the timed steps) and a roofline entry for every instrumented kernel from the
last warm-up step (operator and V-cycle kernels, and the FGMRES Gram-Schmidt
kernels); the FP64-preconditioned GPU solve of the same system (time,
iterations, per-field difference); the other single-GPU workloads (64^3 with
S_eps 0 and 1e-4, the perturbed 96^3 mesh with its adjoint) in FP64; and the
FP64 CPU oracle timed on bounded samples.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# Vector ALU peak of the build: 256 CUs x 64 lanes x 2 flops per fused
# multiply-add x 2.4 GHz = 78.6 TFLOP/s, in FP64 and in FP32 alike (the HIP
# code is compiled without packed FP32 instructions, the only way FP32 vector
# arithmetic reaches the 157.3 TFLOP/s of the data sheet)
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def _cpu_baseline(sample_n: int, full_unknowns: int):
    """The FP64 oracle as it stands, on the host's cores (BLAS threads up to
    16, the GPU machine's CPU share; SuperLU itself is single-threaded):
    * the 8^3 unit-cube workload: assembly and the direct sparse LU solve that
      defines the step result;
    * the layered workload recipe at sample_n^3: assembly and FGMRES with the
      paper's exact-inner-solve preconditioner M_I^(h), relative residual 1e-8.
    ``value`` projects the second linearly in unknowns to the full workload (a
    lower bound: the sparse LU factorizations grow faster than linearly)."""
    from threadpoolctl import threadpool_limits

    from oracle.solve import BlockPrec, direct_solve, fgmres
    from oracle.system import build_system
    from synth import make_config

    threads = max(1, min(os.cpu_count() or 1, 16))
    with threadpool_limits(threads):
        small = make_config("unit8")
        t0 = time.perf_counter()
        A, b, B = build_system(small)
        direct_solve(A, b)
        t_small = time.perf_counter() - t0
        prob = make_config("layered128", n=sample_n)
        t0 = time.perf_counter()
        A, b, B = build_system(prob)
        t_asm = time.perf_counter() - t0
        P = BlockPrec(B)
        x, its, _ = fgmres(lambda v: A @ v, b, P.apply, rtol=1e-8, restart=200)
        t = time.perf_counter() - t0
    n = prob.n_total
    return {"value": round(t * full_unknowns / n, 3),
            "unit": "s (the layered sample projected linearly in unknowns to the full workload; a lower bound, "
                    "the oracle's sparse LU work grows faster than linearly)",
            "cores": threads, "kind": "oracle",
            "sample": f"layered workload recipe at {sample_n}^3 ({n} unknowns): FP64 assembly + FGMRES with exact "
                      f"inner LU solves (M_I^(h)), rtol 1e-8, {its} iterations",
            "measured": {f"layered{sample_n}": {"seconds": round(t, 3), "assembly_s": round(t_asm, 3),
                                                "unknowns": n, "iterations": its},
                         "unit8": {"seconds": round(t_small, 3), "unknowns": small.n_total,
                                   "what": "8^3 unit cube: FP64 assembly + direct sparse LU of A_H"}}}


def _traffic(kernel: str, n: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary for this workload (FETCH_SIZE + WRITE_SIZE, calibrated on a
    plain copy), or None when there is none or the HIP sources have changed
    since the counters were taken."""
    from paper_2002_09603_amd.profsummary import sources_sha256

    path = os.path.join(ROOT, "profiles", "traffic_layered%d.md" % n)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("TRAFFIC "):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                rec[kv["kernel"]] = kv
    kv = rec.get(kernel.split(" ")[0])
    if kv is None or kv.get("sources_sha256") != sources_sha256():
        return None
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])


def _time_loop_run(args, dev):
    """20 backward-Euler steps on 192 x 192 x 96 cells ([0,2]^2 x [0,1],
    log-normal kappa sigma 3, E = 1e4 exp(0.5 xi), geometric dt 1e-3 -> 1),
    mixed-precision forward and adjoint, loss = sum over steps of the squared
    pressure at 64 observation cells, checkpoints every 5 steps."""
    import torch

    from paper_2002_09603_amd.autograd import time_loop
    from paper_2002_09603_amd.solver import Options, from_problem
    from synth import make_config

    prob = make_config("spe192")
    dts = list(prob.dts)
    print(f"[spe192] {prob.nx}x{prob.ny}x{prob.nz} cells, {prob.n_total} unknowns, {len(dts)} steps", flush=True)
    s = from_problem(prob, Options(rtol=1e-8, rtol_transpose=1e-8, precond_fp32=True, restart=50,
                                   max_it=2000, orth_passes=1), device=dev)
    log = {"solve": [], "solve_transpose": []}
    for name in log:
        fn = getattr(s, name)

        def wrapped(*a, _fn=fn, _rec=log[name], **k):
            out = _fn(*a, **k)
            _rec.append(out[-1])
            print(f"   {len(_rec):3d} {_rec is log['solve'] and 'forward' or 'adjoint'} solve: "
                  f"{out[-1]['iters']} its, {out[-1]['t_setup'] + out[-1]['t_solve']:.3f} s", flush=True)
            return out
        setattr(s, name, wrapped)
    logk = torch.tensor(np.log(prob.kappa[:, 0]), dtype=torch.float64, device=dev, requires_grad=True)
    logE = torch.tensor(np.log(prob.E), dtype=torch.float64, device=dev, requires_grad=True)
    obs = torch.as_tensor(prob.obs_cells, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = time_loop(s, logk, logE, dts, every=5)
    loss = (P[:, obs] ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n_fwd = len(dts)
    fwd_its = [i["iters"] for i in log["solve"][:n_fwd]]
    adj_its = [i["iters"] for i in log["solve_transpose"]]
    out = {"metric": "time for the 20-step forward + adjoint run with checkpoints every 5 steps (s)",
           "value": round(t2 - t0, 3), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64 Krylov / f32 preconditioner", "data": "synthetic",
           "config": {"workload": "spe192: 192x192x96 cells on [0,2]^2x[0,1], kappa lognormal sigma 3, "
                                  "E 1e4*lognormal sigma 0.5, nu 0.25, S_eps 0, 20 geometric steps "
                                  "dt 1e-3..1, rtol 1e-8 forward and adjoint",
                      "unknowns": s.N},
           "t_forward_s": round(t1 - t0, 3), "t_backward_s": round(t2 - t1, 3),
           "forward_iterations": fwd_its, "recomputed_forward_solves": len(log["solve"]) - n_fwd,
           "adjoint_iterations": adj_its, "loss": float(loss.detach()),
           "grad_norm": {"dlogk": float(logk.grad.norm()), "dlogE": float(logE.grad.norm())}}
    if args.fd:
        # Directional central difference of the 20-step loss.  Two independent
        # 20-step runs resolve the loss change (~1e-5 of the loss) only to the
        # solver's floor, so each perturbed step solves for its correction to
        # the unperturbed state X_n, A'(theta') d_n = b'_n - A'(theta') X_n, and
        # the loss change is summed as (2 p_n + dp_n) dp_n without cancellation;
        # the perturbed states X_n + d_n still solve the perturbed steps.
        from paper_2002_09603_amd import _capi

        g = torch.Generator(device="cpu").manual_seed(7)
        vk = torch.randn(prob.n_cells, generator=g, dtype=torch.float64).to(dev)
        vE = torch.randn(prob.n_cells, generator=g, dtype=torch.float64).to(dev)
        s.close()
        s = from_problem(prob, Options(rtol=1e-11, precond_fp32=True, restart=50, max_it=3000,
                                       orth_passes=1), device=dev)
        d = args.fd_step
        with torch.no_grad():
            lk, lE = logk.detach(), logE.detach()

            def set_material(lk_, lE_):
                s.update_material(torch.exp(lE_).contiguous(), torch.exp(lk_)[:, None].expand(-1, 3).contiguous())

            def rhs(x_prev):
                if x_prev is None:
                    return s.build_rhs()
                u, p, _ = s.split(x_prev)
                return s.build_rhs(u.contiguous(), p.contiguous())

            set_material(lk, lE)
            X, x = [], None
            for dt in dts:
                s.set_dt(dt)
                u, pi, p, _ = s.solve(rhs(x))
                x = torch.cat([u, p, pi])
                X.append(x)
            dL, worst_corr = [], 0.0
            for sgn in (1.0, -1.0):
                set_material(lk + sgn * d * vk, lE + sgn * d * vE)
                acc, xp = 0.0, None
                for n, dt in enumerate(dts):
                    s.set_dt(dt)
                    du, dpi, dp, inf = s.solve(rhs(xp) - s.apply(_capi.PM_OP_AH, X[n]), raise_noconv=False)
                    worst_corr = max(worst_corr, inf["relres_true"])
                    xp = X[n] + torch.cat([du, dp, dpi])
                    p0 = s.split(X[n])[1][obs]
                    acc += float(((2.0 * p0 + dp[obs]) * dp[obs]).sum())
                dL.append(acc)
        fd = (dL[0] - dL[1]) / (2 * d)
        ad = float((logk.grad * vk).sum() + (logE.grad * vE).sum())
        out["directional_check"] = {"adjoint": ad, "central_difference": fd, "step": d,
                                    "rel_diff": abs(fd - ad) / abs(ad),
                                    "loss_change": {"plus": dL[0], "minus": dL[1]},
                                    "worst_correction_relres": worst_corr}
    s.close()
    print(json.dumps(out), flush=True)


def _cantilever_run(args, dev):
    """The paper's 3D cantilever (unit cube, E 1e5, nu 0.4, kappa 1e-7, mu 1e-3,
    face x = 0 fixed, top loaded, no-flow everywhere) on n^3 cells for
    dt = 0.1 and 1e-5, stopping at a relative residual of 1e-6: iterations and
    times of the hybridized step (eq. stab_A, block upper triangular
    preconditioner) with the translation (separate displacement component)
    and the rigid-body near kernel for A_uu, and of the non-hybridized MFE step
    (eq. mfeSys, block lower triangular preconditioner of eq. prec), the
    comparison of Sec. 5.2 (tables tab:can_1 and tab:can_3)."""
    import torch

    from paper_2002_09603_amd.solver import Options, from_problem
    from synth import cantilever

    runs = []
    for dt in (0.1, 1e-5):
        prob = cantilever(args.n, dt)
        for rbm in (False, True):
            opts = Options(rtol=1e-6, precond_fp32=True, restart=24, max_it=1000, orth_passes=1,
                           cheb_degree_pi=1, cheb_lower_pi=0.1, rbm_u=rbm)
            s = from_problem(prob, opts, device=dev)
            b = torch.empty(s.N, dtype=torch.float64, device=dev)
            best = None
            for rep in range(1 + max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.assemble()
                s.build_rhs(out=b)
                u, pi, p, info = s.solve(b)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                if rep > 0 and (best is None or t < best[0]):
                    best = (t, info)
            t, info = best
            rec = {"form": "hybrid", "dt": dt, "near_kernel_u": "rigid-body" if rbm else "translations",
                   "iterations": info["iters"], "relres_true": info["relres_true"], "t_total_s": round(t, 4),
                   "t_setup_s": round(info["t_setup"], 4), "t_solve_s": round(info["t_solve"], 4),
                   "amg_levels_u": info["levels_u"], "amg_operator_complexity_u": round(info["opcx_u"], 3)}
            print("   ", json.dumps(rec), flush=True)
            runs.append(rec)
            n_unknowns = s.N
            s.close()
            # the MFE form of the same step, FGMRES(100): restarted every
            # 24 iterations it stagnates at dt = 1e-5 from 64^3 on (its C~_p
            # hierarchy is built on the first call after assembly).  Its two
            # Krylov bases (2 x 101 vectors of N doubles) take 191 GB at 256^3,
            # more than the device has beside the operators: skipped there.
            mfe_bases = 2 * 101 * n_unknowns * 8
            mfe_room = torch.cuda.get_device_properties(dev).total_memory // 2
            if not rbm and mfe_bases > mfe_room:
                rec = {"form": "mfe", "dt": dt, "skipped": f"FGMRES(100) bases need {mfe_bases / 2**30:.0f} GiB, "
                                                          f"more than half of the device's "
                                                          f"{2 * mfe_room / 2**30:.0f} GiB"}
                print("   ", json.dumps(rec), flush=True)
                runs.append(rec)
            elif not rbm:
                sm = from_problem(prob, dataclasses.replace(opts, restart=100), device=dev)
                bm = torch.empty(sm.N, dtype=torch.float64, device=dev)
                best = None
                for rep in range(1 + max(1, args.steps)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    sm.assemble()
                    sm.build_rhs_mfe(out=bm)
                    u, q, p, info = sm.solve_mfe(bm)
                    torch.cuda.synchronize()
                    t = time.perf_counter() - t0
                    if rep > 0 and (best is None or t < best[0]):
                        best = (t, info)
                t, info = best
                rec = {"form": "mfe", "dt": dt, "near_kernel_u": "translations", "restart": 100,
                       "iterations": info["iters"], "relres_true": info["relres_true"], "t_total_s": round(t, 4),
                       "amg_levels_p": info["levels_pi"]}
                print("   ", json.dumps(rec), flush=True)
                runs.append(rec)
                sm.close()
    first = runs[0]
    out = {"metric": "cantilever: time-to-solution (s) and FGMRES iterations at relres 1e-6",
           "value": first["t_total_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64 Krylov / f32 preconditioner", "data": "synthetic",
           "config": {"workload": f"cantilever{args.n}: {args.n}^3 unit cube, E 1e5, nu 0.4, b 1, S_eps 0, "
                                  "kappa 1e-7, mu 1e-3, x = 0 fixed, top loaded, no-flow everywhere; "
                                  "FGMRES(24), one Gram-Schmidt pass, V(2,2) A_uu, V(1,1) C~pi; MFE form: "
                                  "FGMRES(100) around eq. prec (FP64 V-cycles)",
                      "unknowns": n_unknowns},
           "runs": runs}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="cells per axis of the layered workload")
    ap.add_argument("--cpu-sample", type=int, default=24, help="cells per axis of the oracle sample")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the 64^3 (S_eps 0 and 1e-4) and perturbed 96^3 FP64 solves after the benchmark")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-preconditioned comparison solve")
    ap.add_argument("--rbm", action="store_true",
                    help="rigid-body near kernel (translations and rotations) for the A_uu hierarchy")
    ap.add_argument("--workload", choices=("layered", "spe192", "cantilever"), default="layered",
                    help="layered: one step of the layered workload (the benchmark line); spe192: the "
                         "20-step 192x192x96 forward + adjoint run with checkpoints every 5 steps; "
                         "cantilever: the paper's cantilever on --n^3 cells, translation against "
                         "rigid-body near kernel for A_uu, dt 0.1 and 1e-5")
    ap.add_argument("--fd", action="store_true", help="spe192: also check the gradient against a "
                    "directional central difference (three more 20-step forward runs)")
    ap.add_argument("--fd-step", type=float, default=1e-3, help="step of that central difference in log space")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the steps, run a plain device copy (elementwise negation) that reads and "
                         "writes MIB MiB each, to calibrate HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs (--gpus > 1) are not supported",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_2002_09603_amd import _capi
    from paper_2002_09603_amd.solver import Options, from_problem
    from synth import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "spe192":
        return _time_loop_run(args, dev)
    if args.workload == "cantilever":
        return _cantilever_run(args, dev)
    prob = make_config("layered128", n=args.n)
    # benchmark solver settings: FGMRES(24), one Gram-Schmidt pass, V(2,2) on A_uu,
    # V(1,1) with a wider Chebyshev interval on C~_pi
    opts = Options(rtol=1e-8, precond_fp32=True, restart=24, max_it=1000, orth_passes=1, cheb_degree_pi=1,
                   cheb_lower_pi=0.1, rbm_u=args.rbm)
    s = from_problem(prob, opts, device=dev)
    b = torch.empty(s.N, dtype=torch.float64, device=dev)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def step():
        s.assemble()
        s.build_rhs(out=b)
        u, pi, p, info = s.solve(b)
        w = s.reconstruct_w(p, pi)
        return u, pi, p, w, info

    # warm-up; the last warm-up step records every instrumented kernel: the
    # per-kernel table, and the dominant operator / V-cycle kernel, which the
    # timed steps then record alone
    all_mask = sum(1 << k for k in _capi.PROF_KERNELS)
    for i in range(max(args.warmup, 1)):
        if i == max(args.warmup, 1) - 1:
            s.profile_begin(all_mask)
        step()
    torch.cuda.synchronize()
    totals = {k: s.profile_end(k) for k in _capi.PROF_KERNELS}
    solve_ids = [k for k, (_, role) in _capi.PROF_KERNELS.items() if role == "solve"]
    dom = max(solve_ids, key=lambda k: totals[k][1])
    s.profile_begin(1 << dom)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        u, pi, p, w, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_rec = s.profile_end(dom)
    s.profile_begin(0)
    ms_per_step = 1000.0 * elapsed / args.steps
    last = infos[-1]
    head = _roofline(dom, *dom_rec)
    head["traffic"] = _traffic(_capi.PROF_KERNELS[dom][0], args.n)

    out = {
        "metric": "time-to-solution (s) & FGMRES its at relres 1e-8, 128^3 grid; HBM GB/s of SpMV/V-cycle",
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": None,
        "vs_baseline": None,
        "dtype": "f64 Krylov / f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": f"layered{args.n}: {args.n}^3 hex unit cube, layered anisotropic kappa "
                               "(1e-2,1e-2,1e-6 / 1e-6 in 8-cell layers, lognormal sigma 1), E 1e4, nu 0.25, "
                               "S_eps 0, dt 1e-2; mixed-precision block-triangular AMG preconditioner "
                               "(V(2,2) A_uu, V(1,1) C~pi), FP64 FGMRES(24) with one classical "
                               "Gram-Schmidt pass, rtol 1e-8",
                   "unknowns": s.N, "n_u": s.n_u, "n_pi": s.n_pi, "n_p": s.n_p,
                   "near_kernel_u": "rigid-body (6 modes)" if args.rbm else "translations (3 modes)"},
        "iterations": last["iters"],
        "relres_true": last["relres_true"],
        "t_asm_s": round(last["t_asm"], 4),
        "t_setup_s": round(last["t_setup"], 4),
        "t_solve_s": round(last["t_solve"], 4),
        "amg_levels": [last["levels_u"], last["levels_pi"]],
        "amg_operator_complexity": [round(last["opcx_u"], 3), round(last["opcx_pi"], 3)],
        "roofline": head,
        "kernels_last_warmup": sorted(({**_roofline(k, *v), "traffic": _traffic(_capi.PROF_KERNELS[k][0], args.n)}
                                       for k, v in totals.items() if v[0] > 0), key=lambda e: -e["ms"]),
    }

    if not args.no_fp64:
        s64 = from_problem(prob, Options(rtol=1e-8, precond_fp32=False, restart=24, max_it=1000, orth_passes=1,
                                         cheb_degree_pi=1, cheb_lower_pi=0.1, rbm_u=args.rbm),
                           device=dev)
        s64.assemble()
        b64 = s64.build_rhs()
        s64.solve(b64)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s64.assemble()
        s64.build_rhs(out=b64)
        u64, pi64, p64, i64 = s64.solve(b64)
        s64.reconstruct_w(p64, pi64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1

        def rel(a, r):
            return float(torch.linalg.norm(a - r) / torch.linalg.norm(r))
        out["fp64_precond_solve"] = {
            "time_to_solution_s": round(t64, 4), "iterations": i64["iters"],
            "t_setup_s": round(i64["t_setup"], 4), "t_solve_s": round(i64["t_solve"], 4),
            "mixed_vs_fp64_rel_l2": {"u": rel(u, u64), "p": rel(p, p64), "pi": rel(pi, pi64)}}
        s64.close()
    s.close()

    if not args.no_legs:
        out["other_configs"] = _legs(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(args.cpu_sample, out["config"]["unknowns"])
    print(json.dumps(out), flush=True)


def _roofline(kid, n, ms, by, fl):
    """Roofline entry of one instrumented kernel from its recorded launches:
    against the vector ALU peak when the launches carry stencil flops (the
    matrix-free lattice kernels), else against the HBM peak with the
    algorithmic bytes."""
    from paper_2002_09603_amd import _capi

    label, role = _capi.PROF_KERNELS[kid]
    e = {"kernel": label, "role": role, "launches": n, "ms": round(ms, 3),
         "avg_launch_us": round(1000.0 * ms / max(n, 1), 1),
         "algorithmic_bytes_per_launch": round(by / max(n, 1))}
    if ms <= 0:
        return e
    if fl > 0:
        ach = fl / (ms / 1e3) / 1e12
        e.update({"bound": "alu", "achieved": round(ach, 2), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                  "frac": round(ach / ALU_PEAK_TFLOPS, 4), "flops_per_launch": round(fl / max(n, 1)),
                  "hbm_GB_s": round(by / 1e6 / ms, 1)})
    else:
        ach = by / 1e6 / ms
        e.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ach / HBM_PEAK_GBS, 4)})
    return e


def _legs(dev):
    """The other single-GPU workloads, measured after the benchmark: the 64^3
    cube (log-normal kappa sigma 2, nu 0.3) with S_eps 0 and 1e-4 and the
    perturbed 96^3 mesh (general hexahedra: assembled sliced-ELL A_uu, full
    6x6 M_T^-1) with its adjoint solve and gradient, all in FP64 (FP64 AMG,
    FP64 FGMRES(24), one Gram-Schmidt pass, relative residual 1e-8).  Each is
    timed on a second step after a warm-up step; the per-kernel table comes
    from the timed step."""
    import torch

    from paper_2002_09603_amd import _capi
    from paper_2002_09603_amd.solver import Options, from_problem
    from synth import make_config

    legs = {}
    runs = [("cube64_S0", make_config("cube64", S_eps=0.0)), ("cube64_S1e-4", make_config("cube64", S_eps=1e-4)),
            ("perturbed96", make_config("perturbed96"))]
    all_mask = sum(1 << k for k in _capi.PROF_KERNELS)
    for name, prob in runs:
        s = from_problem(prob, Options(rtol=1e-8, precond_fp32=False, restart=24, max_it=1000, orth_passes=1,
                                       cheb_degree_pi=1, cheb_lower_pi=0.1, rtol_transpose=1e-8), device=dev)
        b = torch.empty(s.N, dtype=torch.float64, device=dev)
        for rep in range(2):
            if rep == 1:
                s.profile_begin(all_mask)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.assemble()
            s.build_rhs(out=b)
            u, pi, p, info = s.solve(b)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        totals = {k: s.profile_end(k) for k in _capi.PROF_KERNELS}
        s.profile_begin(0)
        i = s.info()
        rec = {"unknowns": s.N, "time_to_solution_s": round(t, 4), "iterations": info["iters"],
               "relres_true": info["relres_true"], "t_asm_s": round(info["t_asm"], 4),
               "t_setup_s": round(info["t_setup"], 4), "t_solve_s": round(info["t_solve"], 4),
               "lattice_uu": bool(i["lattice_uu"]), "block_minv": bool(i["block_minv"]),
               "amg_levels": [i["levels_u"], i["levels_pi"]]}
        solve_ids = [k for k, (_, role) in _capi.PROF_KERNELS.items() if role == "solve" and totals[k][0] > 0]
        dom = max(solve_ids, key=lambda k: totals[k][1])
        rec["roofline_dominant_solve_kernel"] = _roofline(dom, *totals[dom])
        rec["kernels"] = sorted((_roofline(k, *v) for k, v in totals.items() if v[0] > 0), key=lambda e: -e["ms"])
        if name == "perturbed96":
            # adjoint of the loss sum of squared pressure at the observation cells
            obs = torch.as_tensor(prob.obs_cells, device=dev)
            g = torch.zeros(s.N, dtype=torch.float64, device=dev)
            g[s.n_u + obs] = 2.0 * p[obs]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lu, lpi, lp, ia = s.solve_transpose(g)
            dk, dE = s.grad(torch.cat([lu, lp, lpi]), torch.cat([u, p, pi]))
            torch.cuda.synchronize()
            rec["adjoint"] = {"time_s": round(time.perf_counter() - t0, 4), "iterations": ia["iters"],
                              "relres_true": ia["relres_true"]}
        print(f"   [{name}] {json.dumps({k: v for k, v in rec.items() if k != 'kernels'})}", file=sys.stderr,
              flush=True)
        legs[name] = rec
        s.close()
    return legs


if __name__ == "__main__":
    main()
