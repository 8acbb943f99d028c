"""Host-side checks of the C ABI library that need no GPU: the library loads,
exports every function include/fepa.h declares, names its status codes, and
rejects invalid set-up arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2112_07075_amd as fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fepa.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fe.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fe.ABI_FUNCTIONS)


def test_status_strings():
    for code in (fe.FE_OK, fe.FE_EINVAL, fe.FE_ENOMEM, fe.FE_EDEVICE, fe.FE_EUNSUPPORTED,
                 fe.FE_EBADMESH, fe.FE_ENOTCONV):
        s = fe.fe_status_str(code)
        assert s and s != "unknown status"
    assert fe.fe_status_str(12345) == "unknown status"


def _desc(E=1, p=2, Q=4, N=27, nodes=None, x0=1):
    D3 = (p + 1) ** 3
    if nodes is None:
        nodes = np.arange(E * D3, dtype=np.int32).reshape(E, D3) % N
    return fe._MeshDesc(E, p, Q, N, nodes.ctypes.data, x0, 1.0), nodes


def _setup(descs, n, opts=None):
    h = C.c_void_p()
    arr = (fe._MeshDesc * max(n, 1))(*descs) if descs else None
    rc = fe.lib().fe_pa_setup(arr, n, C.byref(opts) if opts else None, None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("case,expect", [
    ("no_meshes", fe.FE_EINVAL),
    ("bad_order", fe.FE_EINVAL),
    ("bad_q", fe.FE_EUNSUPPORTED),
    ("map_range", fe.FE_EINVAL),
    ("null_x0", fe.FE_EINVAL),
    ("bad_gamma", fe.FE_EINVAL),
    ("bad_precision", fe.FE_EUNSUPPORTED),
    ("bad_waves", fe.FE_EINVAL),
    ("bad_patch", fe.FE_EINVAL),
    ("unknown_flag", fe.FE_EINVAL),
    ("zero_rho0", fe.FE_EINVAL),
    ("rho0_q_with_materials", fe.FE_EUNSUPPORTED),
])
def test_setup_rejects_invalid_arguments_without_device(case, expect):
    d, keep = _desc()
    opts = None
    n = 1
    if case == "no_meshes":
        n = 0
    elif case == "bad_order":
        d.order = 7
    elif case == "bad_q":
        d.q1d = 9
    elif case == "map_range":
        keep[0, 3] = 27
    elif case == "null_x0":
        d.x0 = None
    elif case == "bad_gamma":
        opts = fe._Opts(0, 0, 0.5, 0.5, 2.0, 0, 0, 0, 0)
    elif case == "bad_precision":
        opts = fe._Opts(7, 0, 5.0 / 3.0, 0.5, 2.0, 0, 0, 0, 0)
    elif case == "bad_waves":
        opts = fe._Opts(0, 0, 5.0 / 3.0, 0.5, 2.0, 3, 0, 0, 0)
    elif case == "bad_patch":
        opts = fe._Opts(0, 0, 5.0 / 3.0, 0.5, 2.0, 0, 0, 0, 5000)
    elif case == "unknown_flag":
        opts = fe._Opts(0, 0x40, 5.0 / 3.0, 0.5, 2.0, 0, 0, 0, 0)
    elif case == "zero_rho0":
        d.rho0 = 0.0  # and no per-point density
    elif case == "rho0_q_with_materials":
        # both checked on the host, before any device work: the pointers are
        # never read
        d.rho0_q = 0x1000
        g, r = (C.c_double * 1)(1.4), (C.c_double * 1)(1.0)
        keep = (keep, g, r)
        mat = fe._Materials(1, C.cast(g, C.c_void_p), C.cast(r, C.c_void_p), 0x2000)
        opts = fe._Opts(0, 0, 5.0 / 3.0, 0.5, 2.0, 0, 0, 0, 0, None, C.pointer(mat))
    rc, h = _setup([d], n, opts)
    assert rc == expect
    assert not h.value
    assert fe.lib().fe_last_error(None).decode()


def test_null_context_calls():
    L = fe.lib()
    assert L.fe_query(None, None) == fe.FE_EINVAL
    assert L.fe_qdata_update(None, None, None, None) == fe.FE_EINVAL
    assert L.fe_force_mult(None, None, None) == fe.FE_EINVAL
    assert L.fe_force_mult_T(None, None, None) == fe.FE_EINVAL
    assert L.fe_force_mult_pair(None, None, None, None, None) == fe.FE_EINVAL
    assert L.fe_force_mult_pair_noalloc(None, None, None, None, None) == fe.FE_EINVAL
    assert L.fe_mass_mult(None, None, None) == fe.FE_EINVAL
    assert L.fe_mass_cg(None, None, None, None, 0, 1e-12, 10, None, None) == fe.FE_EINVAL
    assert L.fe_get_diag(None, None) == fe.FE_EINVAL
    assert L.fe_export_qdata(None, None, None) == fe.FE_EINVAL
    assert L.fe_timer_reset(None) == fe.FE_EINVAL
    L.fe_destroy(None)


def test_binding_rejects_host_tensors():
    import torch
    with pytest.raises(fe.FepaError):
        fe._ptr(torch.zeros(3))
