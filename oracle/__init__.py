"""ctypes front end of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and
by the benchmark's CPU-baseline leg. The GPU product path never imports it.

Every function takes and returns NumPy float64 / int32 arrays in the layouts of
the synthetic-input module: vectors [3][N] (SoA), L2 fields [E][p^3],
quadrature data S[E][3][3][Q^3] and m_q[E][Q^3].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_vp = C.c_void_p


def build() -> str:
    """Compile oracle.c with gcc (-O2, no FMA contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall",
           "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.or_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.or_gll_nodes.argtypes = [C.c_int, _dp]
        L.or_lagrange.argtypes = [C.c_int, _dp, C.c_double, _dp, _dp]
        L.or_lagrange.restype = None
        L.or_qdata.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _dp, _vp, _vp,
                               C.c_double, C.c_double, C.c_double, C.c_double, _vp, C.c_int,
                               _vp, _vp, _vp]
        L.or_force_elem_matrix.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_mass_elem_matrix.argtypes = [C.c_int, C.c_int, _dp, _dp]
        for fn in (L.or_force_mult, L.or_force_mult_T, L.or_mass_mult):
            fn.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _vp, _vp, C.c_int,
                           C.c_int, _dp]
        L.or_mass_cg.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _dp, _dp, _vp,
                                 C.c_int, C.c_double, C.c_int, C.POINTER(C.c_int),
                                 C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ 1-D rules
def gauss_legendre(n: int):
    t, w = np.zeros(n), np.zeros(n)
    if lib().or_gauss_legendre(n, t, w):
        raise ValueError(n)
    return t, w


def gll_nodes(p: int):
    t = np.zeros(p + 1)
    if lib().or_gll_nodes(p, t):
        raise ValueError(p)
    return t


def lagrange(nodes, x: float):
    nodes = _f64(nodes)
    val, der = np.zeros(len(nodes)), np.zeros(len(nodes))
    lib().or_lagrange(len(nodes), nodes, float(x), val, der)
    return val, der


# ------------------------------------------------------------------ operators
class OracleError(RuntimeError):
    pass


def qdata(mesh_map, p, Q, N, x0, x, v, e, rho0=1.0, gamma=5.0 / 3.0, q1=0.5, q2=2.0,
          elems=None, want=("S", "mq", "detJ"), allow_bad=False):
    """Quadrature data: dict with S [E][3][3][Q^3], mq [E][Q^3], detJ [E][Q^3]."""
    mesh_map = _i32(mesh_map)
    E = mesh_map.shape[0]
    Q3 = Q ** 3
    out = {k: np.zeros((E, 9 * Q3) if k == "S" else (E, Q3)) for k in want}
    x0, x, v, e = _f64(x0), _f64(x), _f64(v), _f64(e)
    el = _i32(elems)
    rc = lib().or_qdata(E, p, Q, N, mesh_map, x0, x, _ptr(v), _ptr(e), rho0, gamma, q1, q2,
                        _ptr(el), 0 if el is None else len(el),
                        _ptr(out.get("S")), _ptr(out.get("mq")), _ptr(out.get("detJ")))
    if rc == -2 and not allow_bad:
        raise OracleError("non-positive Jacobian determinant")
    if rc not in (0, -2):
        raise OracleError(f"or_qdata failed: {rc}")
    if "S" in out:
        out["S"] = out["S"].reshape(E, 3, 3, Q3)
    return out


def force_elem_matrix(p, Q, S_el):
    D3, Dl3 = (p + 1) ** 3, p ** 3
    FE = np.zeros(3 * D3 * Dl3)
    lib().or_force_elem_matrix(p, Q, _f64(S_el).ravel(), FE)
    return FE.reshape(3, D3, Dl3)


def mass_elem_matrix(p, Q, mq_el):
    D3 = (p + 1) ** 3
    ME = np.zeros(D3 * D3)
    lib().or_mass_elem_matrix(p, Q, _f64(mq_el).ravel(), ME)
    return ME.reshape(D3, D3)


def force_mult(mesh_map, p, Q, N, S, e=None, elems=None, absmode=False):
    """y = F e ([3][N]); e=None means e = 1."""
    mesh_map = _i32(mesh_map)
    y = np.zeros(3 * N)
    el = _i32(elems)
    rc = lib().or_force_mult(mesh_map.shape[0], p, Q, N, mesh_map, _f64(S).ravel(),
                             _ptr(_f64(e)), _ptr(el), 0 if el is None else len(el),
                             int(absmode), y)
    if rc:
        raise OracleError(f"or_force_mult failed: {rc}")
    return y.reshape(3, N)


def force_mult_T(mesh_map, p, Q, N, S, v, elems=None, absmode=False):
    """z = F^T v ([E][p^3]); rows of unselected elements are left zero."""
    mesh_map = _i32(mesh_map)
    E = mesh_map.shape[0]
    z = np.zeros(E * p ** 3)
    el = _i32(elems)
    rc = lib().or_force_mult_T(E, p, Q, N, mesh_map, _f64(S).ravel(), _ptr(_f64(v)),
                               _ptr(el), 0 if el is None else len(el), int(absmode), z)
    if rc:
        raise OracleError(f"or_force_mult_T failed: {rc}")
    return z.reshape(E, p ** 3)


def mass_mult(mesh_map, p, Q, N, mq, x, elems=None, absmode=False):
    """y = M_v x ([3][N])."""
    mesh_map = _i32(mesh_map)
    y = np.zeros(3 * N)
    el = _i32(elems)
    rc = lib().or_mass_mult(mesh_map.shape[0], p, Q, N, mesh_map, _f64(mq).ravel(),
                            _ptr(_f64(x)), _ptr(el), 0 if el is None else len(el),
                            int(absmode), y)
    if rc:
        raise OracleError(f"or_mass_mult failed: {rc}")
    return y.reshape(3, N)


def mass_cg(mesh_map, p, Q, N, mq, b, x0=None, ess=None, rel_tol=1e-12, max_iter=1000):
    """CG on M_v x = b with x = 0 on ess; returns (x [3][N], iters, rel_res, converged)."""
    mesh_map = _i32(mesh_map)
    x = np.zeros(3 * N) if x0 is None else _f64(x0).ravel().copy()
    es = _i32(ess)
    it, rr = C.c_int(0), C.c_double(0.0)
    rc = lib().or_mass_cg(mesh_map.shape[0], p, Q, N, mesh_map, _f64(mq).ravel(),
                          _f64(b).ravel(), x, _ptr(es), 0 if es is None else len(es),
                          rel_tol, max_iter, C.byref(it), C.byref(rr))
    if rc < 0:
        raise OracleError(f"or_mass_cg failed: {rc}")
    return x.reshape(3, N), it.value, rr.value, rc == 0
