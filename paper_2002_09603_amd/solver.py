"""Python face of the C ABI: a thin object wrapper that marshals torch device
tensors (or host arrays) into ``pm_*`` calls.  All arithmetic runs in the HIP
library; this module only allocates output tensors and passes pointers and
the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _capi
from ._capi import check, lib


def _ptr(t) -> Optional[int]:
    """Pointer of a set-up input (the library copies these with
    hipMemcpyDefault, so host arrays are allowed here)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        if t.dtype != np.float64 or not t.flags.c_contiguous:
            raise ValueError("expected a C-contiguous float64 array")
        return t.ctypes.data
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 tensor")
    return t.data_ptr()


def _dev_f64(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=device)


@dataclass
class Options:
    rtol: float = 1e-8
    restart: int = 100
    max_it: int = 1000
    precond_fp32: bool = False
    stabilize: bool = True
    increment_stab: bool = True
    cheb_degree: int = 2
    coarse_max: int = 64
    cheb_degree_pi: int = 2
    cycles_u: int = 1
    cycles_pi: int = 1
    orth_passes: int = 2
    theta_u: float = 0.0
    theta_pi: float = 0.08
    agg_dist_u: int = 2
    agg_dist_pi: int = 2
    cheb_lower: float = 0.3
    rtol_transpose: float = 0.0
    restart_transpose: int = 100
    orth_passes_transpose: int = 2
    lattice_uu: bool = True
    p_trunc_pi: float = 0.02
    cell_pi: bool = True
    p_trunc_u: float = 0.02
    cheb_lower_pi: float = 0.0
    block_minv: bool = True
    rbm_u: bool = False

    def to_c(self) -> _capi.pm_opts:
        o = _capi.pm_opts()
        o.rtol = self.rtol
        o.restart = self.restart
        o.max_it = self.max_it
        o.precond_fp32 = int(self.precond_fp32)
        o.stabilize = int(self.stabilize)
        o.increment_stab = int(self.increment_stab)
        o.cheb_degree = self.cheb_degree
        o.coarse_max = self.coarse_max
        o.cheb_degree_pi = self.cheb_degree_pi
        o.cycles_u = self.cycles_u
        o.cycles_pi = self.cycles_pi
        o.orth_passes = self.orth_passes
        o.theta_u = self.theta_u
        o.theta_pi = self.theta_pi
        o.agg_dist_u = self.agg_dist_u
        o.agg_dist_pi = self.agg_dist_pi
        o.cheb_lower = self.cheb_lower
        o.rtol_transpose = self.rtol_transpose
        o.restart_transpose = self.restart_transpose
        o.orth_passes_transpose = self.orth_passes_transpose
        o.lattice_uu = int(self.lattice_uu)
        o.p_trunc_pi = self.p_trunc_pi
        o.cell_pi = int(self.cell_pi)
        o.p_trunc_u = self.p_trunc_u
        o.cheb_lower_pi = self.cheb_lower_pi
        o.block_minv = int(self.block_minv)
        o.rbm_u = int(self.rbm_u)
        return o


class PoroSolver:
    """One hybridized poromechanics step on one GPU (see include/poromech.h).

    ``coords`` (n_nodes x 3, or None for a uniform box of size ``L``),
    ``E`` (n_cells), ``kappa`` (n_cells x 3): numpy arrays or tensors.
    """

    def __init__(self, nx, ny, nz, E, kappa, coords=None, L=(1.0, 1.0, 1.0), nu=0.25, biot=1.0,
                 S_eps=0.0, mu=1.0, dt=1e-2, traction=(0.0, 0.0, -1.0), p_top=0.0, rollers=False,
                 opts: Optional[Options] = None, device="cuda", cantilever=False):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.material_version = 0   # bumped by every call that replaces E or kappa
        self.opts = opts or Options()
        self.dt = float(dt)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        E_d = _dev_f64(E, self.device).reshape(-1)
        k_d = _dev_f64(kappa, self.device).reshape(-1)
        X_d = None if coords is None else _dev_f64(coords, self.device).reshape(-1)
        nc = self.nx * self.ny * self.nz
        nn = (self.nx + 1) * (self.ny + 1) * (self.nz + 1)
        for t, n, name in ((E_d, nc, "E"), (k_d, 3 * nc, "kappa"), (X_d, 3 * nn, "coords")):
            if t is not None and t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} values, {n} expected")
        mesh = _capi.pm_mesh(self.nx, self.ny, self.nz, _ptr(X_d), float(L[0]), float(L[1]), float(L[2]))
        mat = _capi.pm_material(_ptr(E_d), _ptr(k_d), float(nu), float(biot), float(S_eps), float(mu))
        kind = (_capi.PM_BC_CANTILEVER if cantilever else
                (_capi.PM_BC_ROLLERS if rollers else _capi.PM_BC_COLUMN))
        bc = _capi.pm_bc((C.c_double * 3)(*[float(t) for t in traction]), float(p_top), kind)
        o = self.opts.to_c()
        self._ctx = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = lib.pm_setup(C.byref(mesh), C.byref(mat), C.byref(bc), float(dt), C.byref(o), C.c_void_p(stream),
                          C.byref(self._ctx))
        if rc != _capi.PM_OK:
            raise _capi.PMError(rc, lib.pm_last_error(None).decode())
        sz = (C.c_int64 * 6)()
        check(lib.pm_sizes(self._ctx, sz), self._ctx)
        self.n_u, self.n_p, self.n_pi, self.N, self.n_nodes, self.n_macro = [int(v) for v in sz]

    # -- lifecycle -------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.pm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def _dev(self, t, n, name, optional=False) -> Optional[int]:
        """Pointer of a vector handed to a device kernel: a contiguous float64
        tensor on this solver's device with exactly n elements (the kernels
        read and write it without bounds of their own)."""
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch tensor on {self.device}, got {type(t).__name__}")
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, the solver on {self.device}")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, {n} expected")
        return t.data_ptr()

    # -- C ABI calls -------------------------------------------------------------
    def assemble(self):
        check(lib.pm_assemble(self._ctx), self._ctx)
        self.material_version += 1
        return self

    def set_dt(self, dt):
        """Change dt (rebuilds C~_pi and its hierarchy); no-op if unchanged."""
        if float(dt) == self.dt:
            return
        check(lib.pm_set_dt(self._ctx, float(dt)), self._ctx)
        self.dt = float(dt)

    def update_material(self, E=None, kappa=None):
        E_d = None if E is None else _dev_f64(E, self.device).reshape(-1)
        k_d = None if kappa is None else _dev_f64(kappa, self.device).reshape(-1)
        if E_d is not None and E_d.numel() != self.n_p:
            raise ValueError(f"E has {E_d.numel()} values, {self.n_p} expected")
        if k_d is not None and k_d.numel() != 3 * self.n_p:
            raise ValueError(f"kappa has {k_d.numel()} values, {3 * self.n_p} expected")
        self.material_version += 1
        check(lib.pm_update_material(self._ctx, _ptr(E_d), _ptr(k_d)), self._ctx)

    def build_rhs(self, u_prev=None, p_prev=None, out=None):
        b = self._empty(self.N) if out is None else out
        check(lib.pm_build_rhs(self._ctx, self._dev(u_prev, self.n_u, "u_prev", True),
                               self._dev(p_prev, self.n_p, "p_prev", True), self._dev(b, self.N, "out")),
              self._ctx)
        return b

    def _solve(self, fn, b, raise_noconv):
        u, pi, p = self._empty(self.n_u), self._empty(self.n_pi), self._empty(self.n_p)
        info = _capi.pm_info()
        rc = fn(self._ctx, self._dev(b, self.N, "right-hand side"), _ptr(u), _ptr(pi), _ptr(p), C.byref(info))
        if rc != _capi.PM_OK and (rc != _capi.PM_ENOCONV or raise_noconv):
            check(rc, self._ctx)
        d = info.as_dict()
        d["converged"] = rc == _capi.PM_OK
        return u, pi, p, d

    def solve(self, b, raise_noconv=True):
        """A_H x = b -> (u, pi, p, info)."""
        return self._solve(lib.pm_solve, b, raise_noconv)

    def build_rhs_mfe(self, u_prev=None, p_prev=None, out=None):
        """[f_u; f_q; f_p] of the MFE form of the step (order [u; q; p])."""
        b = self._empty(self.N) if out is None else out
        check(lib.pm_build_rhs_mfe(self._ctx, self._dev(u_prev, self.n_u, "u_prev", True),
                                   self._dev(p_prev, self.n_p, "p_prev", True), self._dev(b, self.N, "out")),
              self._ctx)
        return b

    def solve_mfe(self, b, raise_noconv=True):
        """A_M x = b (MFE form, block triangular preconditioner) -> (u, q, p, info)."""
        u, q, p = self._empty(self.n_u), self._empty(self.n_pi), self._empty(self.n_p)
        info = _capi.pm_info()
        rc = lib.pm_solve_mfe(self._ctx, self._dev(b, self.N, "right-hand side"), _ptr(u), _ptr(q), _ptr(p),
                              C.byref(info))
        if rc != _capi.PM_OK and (rc != _capi.PM_ENOCONV or raise_noconv):
            check(rc, self._ctx)
        d = info.as_dict()
        d["converged"] = rc == _capi.PM_OK
        return u, q, p, d

    def solve_noalloc(self, b, u, pi, p, raise_noconv=True):
        """A_H x = b into the caller's u, pi, p through pm_solve_noalloc (no
        device allocation in the library; workspace in its static scratch)."""
        info = _capi.pm_info()
        rc = lib.pm_solve_noalloc(self._ctx, self._dev(b, self.N, "right-hand side"), self._dev(u, self.n_u, "u"),
                                  self._dev(pi, self.n_pi, "pi"), self._dev(p, self.n_p, "p"), C.byref(info))
        if rc != _capi.PM_OK and (rc != _capi.PM_ENOCONV or raise_noconv):
            check(rc, self._ctx)
        d = info.as_dict()
        d["converged"] = rc == _capi.PM_OK
        return d

    def solve_transpose(self, g, raise_noconv=True):
        """A_H^T lam = g -> (lam_u, lam_pi, lam_p, info)."""
        return self._solve(lib.pm_solve_transpose, g, raise_noconv)

    def grad(self, lam, x, p_prev=None, dlogk=None, dlogE=None):
        dk = torch.zeros(self.n_p, dtype=torch.float64, device=self.device) if dlogk is None else dlogk
        dE = torch.zeros(self.n_p, dtype=torch.float64, device=self.device) if dlogE is None else dlogE
        check(lib.pm_grad(self._ctx, self._dev(lam, self.N, "lam"), self._dev(x, self.N, "x"),
                          self._dev(p_prev, self.n_p, "p_prev", True), self._dev(dk, self.n_p, "dlogk"),
                          self._dev(dE, self.n_p, "dlogE")), self._ctx)
        return dk, dE

    def rhs_adjoint(self, lam, c):
        check(lib.pm_rhs_adjoint(self._ctx, self._dev(lam, self.N, "lam"), self._dev(c, self.N, "c")), self._ctx)
        return c

    def reconstruct_w(self, p, pi):
        w = self._empty(6 * self.n_p)
        check(lib.pm_reconstruct_w(self._ctx, self._dev(p, self.n_p, "p"), self._dev(pi, self.n_pi, "pi"), _ptr(w)),
              self._ctx)
        return w.view(self.n_p, 6)

    def op_sizes(self, which):
        """(input length, output length) of pm_apply's operator ``which``."""
        sizes = {_capi.PM_OP_CPI: (self.n_pi, self.n_pi), _capi.PM_OP_BP: (self.n_p, self.n_p),
                 _capi.PM_OP_CP: (self.n_p, self.n_p), _capi.PM_OP_VCYCLE_CP: (self.n_p, self.n_p),
                 _capi.PM_OP_AUU: (self.n_u, self.n_u), _capi.PM_OP_VCYCLE_U: (self.n_u, self.n_u),
                 _capi.PM_OP_VCYCLE_PI: (self.n_pi, self.n_pi)}
        if which in sizes:
            return sizes[which]
        if which in (_capi.PM_OP_AH, _capi.PM_OP_AHT, _capi.PM_OP_MINV, _capi.PM_OP_MINVT, _capi.PM_OP_MFE,
                     _capi.PM_OP_BTP):
            return self.N, self.N
        raise ValueError(f"unknown operator {which}")

    def apply(self, which, x):
        n_in, n_out = self.op_sizes(which)
        y = self._empty(n_out)
        check(lib.pm_apply(self._ctx, int(which), self._dev(x, n_in, "x"), _ptr(y)), self._ctx)
        return y

    def profile_begin(self, mask):
        check(lib.pm_profile_begin(self._ctx, int(mask)), self._ctx)

    def profile_end(self, kernel_id):
        """(launches, summed ms, summed algorithmic bytes, summed stencil flops) of one kernel id."""
        n, ms, by, fl = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        check(lib.pm_profile_end(self._ctx, int(kernel_id), C.byref(n), C.byref(ms), C.byref(by), C.byref(fl)),
              self._ctx)
        return int(n.value), float(ms.value), float(by.value), float(fl.value)

    def info(self):
        i = _capi.pm_info()
        check(lib.pm_get_info(self._ctx, C.byref(i)), self._ctx)
        return i.as_dict()

    def pack(self, u, p, pi):
        return torch.cat([u, p, pi])

    def split(self, x):
        return x[:self.n_u], x[self.n_u:self.n_u + self.n_p], x[self.n_u + self.n_p:]


def from_problem(prob, opts: Optional[Options] = None, device="cuda") -> PoroSolver:
    """Build a solver from a ``synth.Problem``-like object (attributes only)."""
    return PoroSolver(prob.nx, prob.ny, prob.nz, prob.E, prob.kappa, coords=prob.coords, nu=prob.nu,
                      biot=prob.biot, S_eps=prob.S_eps, mu=prob.mu, dt=prob.dt, traction=prob.traction,
                      p_top=prob.p_top, rollers=getattr(prob, "rollers", False),
                      opts=opts or Options(stabilize=getattr(prob, "stabilize", True)), device=device,
                      cantilever=getattr(prob, "bc", "column") == "cantilever")
