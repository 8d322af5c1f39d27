"""ctypes declarations of the C ABI in include/poromech.h (argument
marshalling only; every step of the computation runs in the HIP library).

Importing this module loads ``libporomech.so`` from the package directory and
raises ``ImportError`` if it has not been built (``__graft_entry__.build()``
or ``python paper_2002_09603_amd/build.py``).  There is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libporomech.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EHIP, PM_ENOCONV, PM_EBREAKDOWN, PM_ESTATE, PM_EINTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7
PM_BC_COLUMN, PM_BC_ROLLERS, PM_BC_CANTILEVER = 0, 1, 2
PM_OP_AH, PM_OP_AHT, PM_OP_MINV, PM_OP_MINVT, PM_OP_CPI, PM_OP_BP, PM_OP_AUU, \
    PM_OP_VCYCLE_U, PM_OP_VCYCLE_PI, PM_OP_MFE, PM_OP_CP, \
    PM_OP_VCYCLE_CP, PM_OP_BTP = range(13)

# kernel ids of pm_profile_begin / pm_profile_end: (label, role); role "solve"
# marks the operator, smoother and transfer kernels of the preconditioned
# operator (SpMV and V-cycle), "krylov" the Gram-Schmidt kernels of FGMRES
PROF_KERNELS = {1: ("k_lat_ah_u|k_ah_u (u-rows of A_H, FP64)", "solve"),
                2: ("k_lat_cheb|k_cheb_step<3> (Chebyshev step, finest A_uu level)", "solve"),
                3: ("k_cp_cheb|k_cheb_step<1> (Chebyshev step, finest C~pi level)", "solve"),
                4: ("k_multidot (Gram-Schmidt projections)", "krylov"),
                5: ("k_orth_normalize_n<NG>|k_orth_normalize|k_multiaxpy (Gram-Schmidt update of the new basis vector)",
                    "krylov"),
                6: ("k_residual_csr<3> (restriction from the finest A_uu level)", "solve"),
                7: ("k_ah_p (p-rows of A_H)", "solve"),
                8: ("k_ah_pi_block|k_ah_pi (pi-rows of A_H)", "solve"),
                9: ("k_sell_apply<3> (prolongation onto the finest A_uu level)", "solve"),
                10: ("k_residual_csr<1> (restriction from the finest C~pi level)", "solve"),
                11: ("k_sell_apply<1> (prolongation onto the finest C~pi level)", "solve"),
                12: ("k_lat_residual (residual on the finest A_uu level)", "solve"),
                13: ("k_cp_residual (residual on the finest C~pi level)", "solve")}

ERROR_NAMES = {PM_EINVAL: "PM_EINVAL", PM_ENOMEM: "PM_ENOMEM", PM_EHIP: "PM_EHIP",
               PM_ENOCONV: "PM_ENOCONV", PM_EBREAKDOWN: "PM_EBREAKDOWN",
               PM_ESTATE: "PM_ESTATE", PM_EINTERNAL: "PM_EINTERNAL"}


class pm_mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("coords", C.c_void_p), ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double)]


class pm_material(C.Structure):
    _fields_ = [("E", C.c_void_p), ("kappa", C.c_void_p), ("nu", C.c_double), ("biot", C.c_double),
                ("S_eps", C.c_double), ("mu", C.c_double)]


class pm_bc(C.Structure):
    _fields_ = [("traction_top", C.c_double * 3), ("p_top", C.c_double), ("kind", C.c_int32)]


class pm_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_it", C.c_int32),
                ("precond_fp32", C.c_int32), ("stabilize", C.c_int32), ("increment_stab", C.c_int32),
                ("cheb_degree", C.c_int32), ("coarse_max", C.c_int32),
                ("cheb_degree_pi", C.c_int32), ("cycles_u", C.c_int32), ("cycles_pi", C.c_int32),
                ("orth_passes", C.c_int32),
                ("theta_u", C.c_double), ("theta_pi", C.c_double),
                ("agg_dist_u", C.c_int32), ("agg_dist_pi", C.c_int32), ("cheb_lower", C.c_double),
                ("rtol_transpose", C.c_double), ("restart_transpose", C.c_int32),
                ("orth_passes_transpose", C.c_int32), ("lattice_uu", C.c_int32),
                ("p_trunc_pi", C.c_double), ("cell_pi", C.c_int32), ("p_trunc_u", C.c_double),
                ("cheb_lower_pi", C.c_double), ("block_minv", C.c_int32),
                ("rbm_u", C.c_int32)]


class pm_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("levels_u", C.c_int32), ("levels_pi", C.c_int32),
                ("relres_est", C.c_double), ("relres_true", C.c_double),
                ("t_asm", C.c_double), ("t_setup", C.c_double), ("t_solve", C.c_double),
                ("opcx_u", C.c_double), ("opcx_pi", C.c_double), ("lattice_uu", C.c_int32),
                ("block_minv", C.c_int32), ("ncoarse_u", C.c_int32), ("ncoarse_pi", C.c_int32),
                ("lattice_form", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes)
_SIGS = [
    ("pm_default_opts", None, [C.POINTER(pm_opts)]),
    ("pm_setup", C.c_int, [C.POINTER(pm_mesh), C.POINTER(pm_material), C.POINTER(pm_bc), C.c_double,
                           C.POINTER(pm_opts), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("pm_assemble", C.c_int, [C.c_void_p]),
    ("pm_set_dt", C.c_int, [C.c_void_p, C.c_double]),
    ("pm_update_material", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_build_rhs", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(pm_info)]),
    ("pm_solve_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(pm_info)]),
    ("pm_build_rhs_mfe", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_solve_mfe", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(pm_info)]),
    ("pm_solve_transpose", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(pm_info)]),
    ("pm_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_rhs_adjoint", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_reconstruct_w", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pm_apply", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pm_profile_begin", C.c_int, [C.c_void_p, C.c_uint32]),
    ("pm_profile_end", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("pm_sizes", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("pm_get_info", C.c_int, [C.c_void_p, C.POINTER(pm_info)]),
    ("pm_last_error", C.c_char_p, [C.c_void_p]),
    ("pm_destroy", None, [C.c_void_p]),
]

EXPORTED = [s[0] for s in _SIGS]


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, res, args in _SIGS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = load()


class PMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc, ctx=None):
    if rc != PM_OK:
        msg = lib.pm_last_error(ctx)
        raise PMError(rc, msg.decode() if msg else "")
    return rc


def default_opts() -> pm_opts:
    o = pm_opts()
    lib.pm_default_opts(C.byref(o))
    return o
