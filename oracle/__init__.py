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
                               _vp, _vp, _vp, _vp]
        L.or_qdata_pt.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _dp, _vp, _vp,
                                  C.c_double, _vp, C.c_double, C.c_double, C.c_double, _vp,
                                  C.c_int, _vp, _vp, _vp, _vp]
        L.or_l2_mass.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp]
        L.or_force_elem_matrix.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_mass_elem_matrix.argtypes = [C.c_int, C.c_int, _dp, _dp]
        for fn in (L.or_force_mult, L.or_force_mult_T, L.or_mass_mult):
            fn.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _vp, _vp, C.c_int,
                           C.c_int, _dp]
        L.or_qdata_mm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, C.c_int, _dp, _dp, _dp,
                                  _dp, _dp, _dp, _dp, C.c_double, C.c_double, _dp, _vp]
        L.or_stiff_elem_matrix.argtypes = [C.c_int, C.c_int, C.c_int, _ip, _dp, _vp, _dp]
        L.or_stiff_mult.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _vp, _dp, _vp,
                                    C.c_int, C.c_int, _dp]
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
    """Quadrature data: dict with S [E][3][3][Q^3], mq, detJ and dt (the per-point
    stable time step) [E][Q^3], as asked for in want. rho0 is the initial
    density: a number, or an [E][Q^3] array of its value at every point."""
    mesh_map = _i32(mesh_map)
    E = mesh_map.shape[0]
    Q3 = Q ** 3
    out = {k: np.zeros((E, 9 * Q3) if k == "S" else (E, Q3)) for k in want}
    x0, x, v, e = _f64(x0), _f64(x), _f64(v), _f64(e)
    el = _i32(elems)
    r0q = None if np.isscalar(rho0) else _f64(rho0).reshape(E, Q3)
    rc = lib().or_qdata_pt(E, p, Q, N, mesh_map, x0, x, _ptr(v), _ptr(e),
                           1.0 if r0q is not None else float(rho0), _ptr(r0q), gamma, q1, q2,
                           _ptr(el), 0 if el is None else len(el),
                           _ptr(out.get("S")), _ptr(out.get("mq")), _ptr(out.get("detJ")),
                           _ptr(out.get("dt")))
    if rc == -2 and not allow_bad:
        raise OracleError("non-positive Jacobian determinant")
    if rc not in (0, -2):
        raise OracleError(f"or_qdata failed: {rc}")
    if "S" in out:
        out["S"] = out["S"].reshape(E, 3, 3, Q3)
    return out


def qdata_mm(mesh_map, p, Q, N, x0, x, v, e, eta0, gamma, rho0, q1=0.5, q2=2.0, want_mq=False):
    """Multi-material quadrature data: S [K][E][3][3][Q^3] of F_k (eta_k sigma_k),
    from e, eta0 [K][E][p^3] and per-material gamma, rho0 ([K]); with want_mq
    also the material masses per point mqk [K][E][Q^3]. Returns S or (S, mqk)."""
    mesh_map = _i32(mesh_map)
    E = mesh_map.shape[0]
    gamma, rho0 = _f64(np.atleast_1d(gamma)), _f64(np.atleast_1d(rho0))
    K = len(gamma)
    Q3 = Q ** 3
    S = np.zeros(K * E * 9 * Q3)
    mq = np.zeros(K * E * Q3) if want_mq else None
    rc = lib().or_qdata_mm(E, p, Q, N, mesh_map, K, _f64(x0), _f64(x), _f64(v),
                           _f64(e).ravel(), _f64(eta0).ravel(), gamma, rho0, q1, q2, S, _ptr(mq))
    if rc == -2:
        raise OracleError("non-positive Jacobian determinant")
    if rc:
        raise OracleError(f"or_qdata_mm failed: {rc}")
    S = S.reshape(K, E, 3, 3, Q3)
    return (S, mq.reshape(K, E, Q3)) if want_mq else S


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


def stiff_elem_matrix(p, Q, nodes, x, kappa_el=None):
    """Dense element stiffness K_E [D^3][D^3] of the element with node ids `nodes` on positions x."""
    D3 = (p + 1) ** 3
    x = _f64(x)
    KE = np.zeros(D3 * D3)
    rc = lib().or_stiff_elem_matrix(p, Q, x.shape[-1], _i32(nodes), x.ravel(),
                                    _ptr(_f64(kappa_el)), KE)
    if rc:
        raise OracleError(f"or_stiff_elem_matrix failed: {rc}")
    return KE.reshape(D3, D3)


def stiff_mult(mesh_map, p, Q, N, x, u, kappa=None, elems=None, absmode=False):
    """y = K u ([3][N]): the stiffness (diffusion) operator int kappa grad w_i . grad w_j
    on the mesh x, per component; kappa [E][Q^3] or None for 1."""
    mesh_map = _i32(mesh_map)
    y = np.zeros(3 * N)
    el = _i32(elems)
    kap = _f64(kappa)
    rc = lib().or_stiff_mult(mesh_map.shape[0], p, Q, N, mesh_map, _f64(x).ravel(),
                             _ptr(None if kap is None else kap.ravel()), _f64(u).ravel(),
                             _ptr(el), 0 if el is None else len(el), int(absmode), y)
    if rc:
        raise OracleError(f"or_stiff_mult failed: {rc}")
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


# ------------------------------------------------------------ Lagrange step
def l2_mass(mesh_map, p, Q, mq):
    """Element L2 mass matrices M_E [E][p^3][p^3] from m_q (the energy equation's M_E)."""
    E = _i32(mesh_map).shape[0]
    Dl3 = p ** 3
    ME = np.zeros(E * Dl3 * Dl3)
    if lib().or_l2_mass(E, p, Q, _f64(mq).ravel(), ME):
        raise OracleError("or_l2_mass failed")
    return ME.reshape(E, Dl3, Dl3)


def total_energy(mesh_map, p, Q, N, mq, v, e):
    """Kinetic + internal energy: 1/2 v^T M_v v + sum_E 1^T M_E e_E (= int rho e)."""
    kin = 0.5 * float((_f64(v).reshape(3, N) * mass_mult(mesh_map, p, Q, N, mq, v)).sum())
    ME = l2_mass(mesh_map, p, Q, mq)
    inner = float(np.einsum("ejk,ek->", ME, _f64(e).reshape(ME.shape[0], -1)))
    return kin, inner


def lagrange_rhs(mesh_map, p, Q, N, x0, x, v, e, ess, rho0, gamma, q1, q2, cg_tol, vbar=None):
    """Right-hand sides of the semi-discrete system (Sec. 3.3) at one state:
    S from the state, a = M_v^-1 (-F 1) on the free DOFs (0 on ess), and
    de = M_E^-1 F^T w with w = v (or the given vbar). Returns (a, de, dt_min, S)."""
    qd = qdata(mesh_map, p, Q, N, x0, x, v, e, rho0, gamma, q1, q2, want=("S", "mq", "dt"))
    rhs = -force_mult(mesh_map, p, Q, N, qd["S"])
    a, _, _, ok = mass_cg(mesh_map, p, Q, N, qd["mq"], rhs, ess=ess, rel_tol=cg_tol, max_iter=20000)
    if not ok:
        raise OracleError("mass CG did not converge")
    z = force_mult_T(mesh_map, p, Q, N, qd["S"], v if vbar is None else vbar)
    de = np.linalg.solve(l2_mass(mesh_map, p, Q, qd["mq"]), z[:, :, None])[:, :, 0]
    return a, de, float(qd["dt"].min()), qd


def lagrange_step(mesh_map, p, Q, N, x0, x, v, e, ess=None, cfl=0.5, dt_max=np.inf,
                  rho0=1.0, gamma=5.0 / 3.0, q1=0.5, q2=2.0, cg_tol=1e-14):
    """One two-stage step of the semi-discrete Lagrange system (Sec. 3.3):
      M_v dv/dt = -F 1,  M_E de/dt = F^T v,  dx/dt = v.
    The step size is dt = min(dt_max, cfl * min_q dt_q) at the start of the step.
    Stage 1 (midpoint predictor from the state n):
      v_h = v + dt/2 a(n),  e_h = e + dt/2 M_E^-1 F(n)^T v,  x_h = x + dt/2 v.
    Stage 2 (from the midpoint forces):
      v' = v + dt a(h),  vbar = (v + v')/2,  e' = e + dt M_E^-1 F(h)^T vbar,  x' = x + dt vbar.
    Using vbar in both the energy and the position updates makes the change of
    kinetic energy, vbar^T M_v (v' - v) = -dt vbar^T F(h) 1, cancel the change
    of internal energy, dt 1^T F(h)^T vbar, exactly (up to the CG residual).
    Returns (x', v', e', dt)."""
    x, v, e = (_f64(a).copy() for a in (x, v, e))
    a0, de0, dtq, _ = lagrange_rhs(mesh_map, p, Q, N, x0, x, v, e, ess, rho0, gamma, q1, q2, cg_tol)
    dt = min(dt_max, cfl * dtq)
    vh = v + 0.5 * dt * a0
    eh = e + 0.5 * dt * de0
    xh = x + 0.5 * dt * v
    a1, _, _, qd = lagrange_rhs(mesh_map, p, Q, N, x0, xh, vh, eh, ess, rho0, gamma, q1, q2, cg_tol)
    v1 = v + dt * a1
    vbar = 0.5 * (v + v1)
    z = force_mult_T(mesh_map, p, Q, N, qd["S"], vbar)
    de1 = np.linalg.solve(l2_mass(mesh_map, p, Q, qd["mq"]), z[:, :, None])[:, :, 0]
    return x + dt * vbar, v1, e + dt * de1, dt
