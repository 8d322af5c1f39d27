"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/poromech.h declares, has ctypes struct layouts equal to the C ones,
and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "poromech.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2002_09603_amd import _capi
    names = _declared()
    assert "pm_solve" in names and "pm_setup" in names
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pm_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(_capi.EXPORTED) == set(names)


def test_struct_layouts_match_c(tmp_path):
    """sizeof and the offset of every field, C compiler vs. ctypes."""
    from paper_2002_09603_amd import _capi
    structs = [_capi.pm_mesh, _capi.pm_material, _capi.pm_bc, _capi.pm_opts, _capi.pm_info]
    items, want = [], []
    for st in structs:
        items.append(f"sizeof({st.__name__})")
        want.append(C.sizeof(st))
        for name, _ in st._fields_:
            items.append(f"offsetof({st.__name__}, {name})")
            want.append(getattr(st, name).offset)
    body = "".join(f'printf("%zu\\n", (size_t){e});' for e in items)
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "poromech.h"\n'
                   "int main(){" + body + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == want, [(e, g, w) for e, g, w in zip(items, got, want) if g != w]


def test_default_options():
    from paper_2002_09603_amd import _capi
    o = _capi.default_opts()
    assert o.rtol == 1e-8 and o.restart == 100 and o.max_it == 1000 and o.stabilize == 1
    assert o.precond_fp32 == 0 and o.increment_stab == 1 and o.cheb_degree == 2
    assert o.rtol_transpose == 0.0 and o.restart_transpose == 100 and o.orth_passes_transpose == 2
    # direction-block M_T^-1 where the cells allow it; translation-only near kernel for A_uu
    assert o.block_minv == 1 and o.rbm_u == 0 and o.lattice_uu == 1 and o.cell_pi == 1
    assert _capi.PM_BC_CANTILEVER == 2


@pytest.mark.parametrize("dims", [(3, 4, 4), (4, 4, 0), (4, 5, 6)])
def test_setup_rejects_odd_or_empty_dims_without_a_gpu(dims):
    from paper_2002_09603_amd import _capi
    nx, ny, nz = dims
    nc = max(nx * ny * nz, 1)
    E = np.ones(nc)
    k = np.ones((nc, 3))
    mesh = _capi.pm_mesh(nx, ny, nz, None, 1.0, 1.0, 1.0)
    mat = _capi.pm_material(E.ctypes.data, k.ctypes.data, 0.25, 1.0, 0.0, 1.0)
    bc = _capi.pm_bc((C.c_double * 3)(0, 0, -1), 0.0, 0)
    ctx = C.c_void_p()
    rc = _capi.lib.pm_setup(C.byref(mesh), C.byref(mat), C.byref(bc), 1e-2, None, None, C.byref(ctx))
    assert rc == _capi.PM_EINVAL and not ctx.value
    assert b"even" in _capi.lib.pm_last_error(None)


def test_setup_rejects_bad_scalars_without_a_gpu():
    from paper_2002_09603_amd import _capi
    E = np.ones(8)
    k = np.ones((8, 3))
    mesh = _capi.pm_mesh(2, 2, 2, None, 1.0, 1.0, 1.0)
    bc = _capi.pm_bc((C.c_double * 3)(0, 0, -1), 0.0, 0)
    ctx = C.c_void_p()
    for nu, dt in ((0.5, 1e-2), (0.25, 0.0), (-0.1, 1.0)):
        mat = _capi.pm_material(E.ctypes.data, k.ctypes.data, nu, 1.0, 0.0, 1.0)
        rc = _capi.lib.pm_setup(C.byref(mesh), C.byref(mat), C.byref(bc), dt, None, None, C.byref(ctx))
        assert rc == _capi.PM_EINVAL
    # an unknown boundary-condition kind
    mat = _capi.pm_material(E.ctypes.data, k.ctypes.data, 0.25, 1.0, 0.0, 1.0)
    bad = _capi.pm_bc((C.c_double * 3)(0, 0, -1), 0.0, 7)
    assert _capi.lib.pm_setup(C.byref(mesh), C.byref(mat), C.byref(bad), 1e-2, None, None,
                              C.byref(ctx)) == _capi.PM_EINVAL
    assert _capi.lib.pm_assemble(None) == _capi.PM_EINVAL
    assert _capi.lib.pm_solve(None, None, None, None, None, None) == _capi.PM_EINVAL


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    from paper_2002_09603_amd import _capi
    with pytest.raises(ImportError):
        _capi.load(str(tmp_path / "missing.so"))


def test_binding_validates_device_vectors_without_a_gpu():
    """Every vector a kernel reads or writes after set-up must be a contiguous
    float64 tensor on the solver's device with exactly the expected length;
    anything else is a ValueError before any pointer reaches the library."""
    import torch
    from paper_2002_09603_amd.solver import PoroSolver
    s = object.__new__(PoroSolver)
    s.device = torch.device("cpu")
    s.n_u, s.n_p, s.n_pi = 12, 2, 9
    s.N = 23
    ok = torch.zeros(23, dtype=torch.float64)
    assert s._dev(ok, 23, "x") == ok.data_ptr()
    assert s._dev(None, 23, "x", optional=True) is None
    for bad, n in ((np.zeros(23), 23),                                   # host array
                   (torch.zeros(23, dtype=torch.float32), 23),           # wrong dtype
                   (torch.zeros(22, dtype=torch.float64), 23),           # short
                   (torch.zeros(46, dtype=torch.float64)[::2], 23),      # not contiguous
                   (None, 23)):                                          # missing
        with pytest.raises(ValueError):
            s._dev(bad, n, "x")
    # operator input and output lengths of pm_apply
    from paper_2002_09603_amd import _capi
    assert s.op_sizes(_capi.PM_OP_MFE) == (23, 23)
    assert s.op_sizes(_capi.PM_OP_CP) == (2, 2)
    assert s.op_sizes(_capi.PM_OP_VCYCLE_PI) == (9, 9)
    with pytest.raises(ValueError):
        s.op_sizes(99)
