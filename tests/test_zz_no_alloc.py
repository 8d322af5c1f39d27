"""pm_solve_noalloc, the solve entry point for callers that cannot allocate,
through the C ABI: the same FGMRES and preconditioner kernels as pm_solve
with the Krylov workspace in the library's static scratch.

Checked on two calls in a row, the second on a smaller problem (the scratch
still holds the first call's larger contents): the device's free memory is
unchanged by the call, the fields equal pm_solve's bitwise (same kernels,
same launch shapes, deterministic reductions) and match the FP64 oracle's
direct solve to 1e-8 per field; problems or restart lengths beyond the
scratch are rejected with PM_EINVAL before any work."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.solve import direct_solve  # noqa: E402
from oracle.system import build_system, split  # noqa: E402
from paper_2002_09603_amd import _capi  # noqa: E402
from paper_2002_09603_amd.solver import Options, from_problem  # noqa: E402

from gpu_helpers import box_problem, rel  # noqa: E402


def _noalloc(s, b):
    u = torch.empty(s.n_u, dtype=torch.float64, device="cuda")
    pi = torch.empty(s.n_pi, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n_p, dtype=torch.float64, device="cuda")
    info = _capi.pm_info()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rc = _capi.lib.pm_solve_noalloc(s._ctx, C.c_void_p(b.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.c_void_p(pi.data_ptr()), C.c_void_p(p.data_ptr()), C.byref(info))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return rc, u, pi, p, info.as_dict(), free0 - free1


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_solve_equals_pm_solve_on_two_calls(fp32):
    opts = Options(rtol=1e-13, precond_fp32=fp32, restart=24, max_it=2000, orth_passes=1, cheb_degree_pi=1,
                   cheb_lower_pi=0.1)
    for kw in (dict(nx=16, ny=12, nz=8, seed=21), dict(nx=6, ny=4, nz=4, seed=22, perturb=True)):
        prob = box_problem(**kw)
        print(f"[no-alloc solve] {prob.nx}x{prob.ny}x{prob.nz} fp32={fp32}", flush=True)
        A, b_ref, B = build_system(prob)
        x0 = direct_solve(A, b_ref)
        s = from_problem(prob, opts).assemble()
        b = s.build_rhs()
        # first: the no-allocation call, before pm_solve has sized the context's own workspace
        rc, u, pi, p, info, grown = _noalloc(s, b)
        assert rc == _capi.PM_OK, _capi.lib.pm_last_error(s._ctx)
        assert grown == 0
        u2, pi2, p2, info2 = s.solve(b)
        assert info["iters"] == info2["iters"] and info["relres_true"] <= 1e-13
        assert torch.equal(u, u2) and torch.equal(pi, pi2) and torch.equal(p, p2)
        for got, ref in zip((u, p, pi), split(B, x0)):
            assert rel(got.cpu().numpy(), ref) <= 1e-8
        s.close()


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    # restart 64 in FP64 needs 8.3 MB + 129 * 8 B per unknown of the 256 MiB:
    # at most about 252,000 unknowns; 34 x 34 x 32 cells have 272,575
    prob = box_problem(nx=34, ny=34, nz=32, seed=23)
    s = from_problem(prob, Options(rtol=1e-8, restart=64)).assemble()
    b = s.build_rhs()
    rc, *_ = _noalloc(s, b)
    assert rc == _capi.PM_EINVAL
    assert b"exceeds the static scratch" in _capi.lib.pm_last_error(s._ctx)
    s.close()
    small = box_problem(nx=4, ny=4, nz=4, seed=24)
    s = from_problem(small, Options(rtol=1e-8, restart=65)).assemble()
    rc, *_ = _noalloc(s, s.build_rhs())
    assert rc == _capi.PM_EINVAL and b"restart" in _capi.lib.pm_last_error(s._ctx)
    # the context still solves through the allocating entry point
    u, pi, p, info = s.solve(s.build_rhs())
    assert info["converged"]
    s.close()
