"""Python binding of libfepa (MI355X partial-assembly Lagrange-phase operators).

Argument marshalling only: every function forwards torch device pointers and
the current HIP stream to the C ABI of the same name (include/fepa.h). All
arithmetic runs in the library's HIP kernels; there is no fallback path. If
libfepa.so has not been built, every call raises FepaError.

Tensors: H1 vectors are float64 [3][N_tot] (or flat 3*N_tot), L2 vectors are
float64 [E_tot][p^3], all contiguous on the GPU. Meshes are described by
MeshDesc (host int32 element-to-node map, device float64 x0 [3][N]).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfepa.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_EUNSUPPORTED, FE_EBADMESH, FE_ENOTCONV = \
    0, -1, -2, -3, -4, -5, -6
FE_PREC_FP64, FE_PREC_FP32, FE_PREC_BF16 = 0, 1, 2
FE_OPT_TIMERS, FE_OPT_BATCHED, FE_OPT_GRAPH, FE_OPT_STEP, FE_OPT_STIFF, FE_OPT_ATOMIC = \
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20
FE_TIMER_QDATA, FE_TIMER_FORCE, FE_TIMER_FORCE_T, FE_TIMER_MASS, FE_TIMER_PAIR, FE_TIMER_MF = \
    0, 1, 2, 3, 4, 5

ABI_FUNCTIONS = ("fe_pa_setup", "fe_destroy", "fe_query", "fe_mesh_offsets", "fe_qdata_update",
                 "fe_force_mult", "fe_force_mult_T", "fe_force_mult_pair", "fe_mass_mult", "fe_mass_cg",
                 "fe_get_diag", "fe_export_qdata", "fe_timer_read", "fe_timer_reset",
                 "fe_status_str", "fe_last_error", "fe_lagrange_step", "fe_export_l2_mass_inv",
                 "fe_force_mult_pair_noalloc", "fe_stiffness_update", "fe_stiffness_mult",
                 "fe_qdata_update_mm", "fe_force_mult_T_mm", "fe_force_mult_pair_mf")


class FepaError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{status}: {msg}")
        self.status = status


class _MeshDesc(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("order", C.c_int32), ("q1d", C.c_int32),
                ("n_nodes", C.c_int32), ("elem_nodes", C.c_void_p), ("x0", C.c_void_p),
                ("rho0", C.c_double), ("rho0_q", C.c_void_p)]


class _Materials(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("gamma", C.c_void_p), ("rho0", C.c_void_p),
                ("eta0", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("flags", C.c_int32), ("gamma", C.c_double),
                ("q1", C.c_double), ("q2", C.c_double), ("tune_nw_force", C.c_int32),
                ("tune_nw_force_t", C.c_int32), ("tune_nw_mass", C.c_int32),
                ("tune_patch", C.c_int32), ("tune_table", C.c_char_p),
                ("materials", C.POINTER(_Materials))]


class _Info(C.Structure):
    _fields_ = [("n_mesh", C.c_int32), ("nw_force", C.c_int32), ("nw_force_t", C.c_int32),
                ("nw_mass", C.c_int32), ("patch", C.c_int32),
                ("n_elem_total", C.c_int64), ("n_nodes_total", C.c_int64),
                ("l2_size_total", C.c_int64), ("qdata_bytes", C.c_int64),
                ("workspace_bytes", C.c_int64), ("precision", C.c_int32), ("flags", C.c_int32)]


class _Diag(C.Structure):
    _fields_ = [("min_detj", C.c_double), ("nonfinite", C.c_int32), ("cg_iters", C.c_int32),
                ("cg_rel_res", C.c_double), ("dt_est", C.c_double)]


class _StepInfo(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_est", C.c_double), ("cg_iters", C.c_int32 * 2),
                ("cg_rel_res", C.c_double * 2)]


_lib = None


def lib() -> C.CDLL:
    """Load libfepa.so (raises FepaError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FepaError(FE_EDEVICE, f"{LIB_PATH} is missing: build it with "
                                    "`python -m paper_2112_07075_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.fe_pa_setup.argtypes = [C.POINTER(_MeshDesc), i32, C.POINTER(_Opts), vp, C.POINTER(vp)]
    L.fe_destroy.argtypes = [vp]
    L.fe_destroy.restype = None
    L.fe_query.argtypes = [vp, C.POINTER(_Info)]
    L.fe_mesh_offsets.argtypes = [vp, vp, vp, vp]
    L.fe_qdata_update.argtypes = [vp, vp, vp, vp]
    L.fe_force_mult.argtypes = [vp, vp, vp]
    L.fe_force_mult_T.argtypes = [vp, vp, vp]
    L.fe_force_mult_pair.argtypes = [vp, vp, vp, vp, vp]
    L.fe_force_mult_pair_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.fe_stiffness_update.argtypes = [vp, vp, vp]
    L.fe_qdata_update_mm.argtypes = [vp, vp, vp, vp]
    L.fe_force_mult_pair_mf.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fe_force_mult_T_mm.argtypes = [vp, vp, vp]
    L.fe_stiffness_mult.argtypes = [vp, vp, vp]
    L.fe_mass_mult.argtypes = [vp, vp, vp]
    L.fe_mass_cg.argtypes = [vp, vp, vp, vp, i32, dbl, i32, C.POINTER(i32), C.POINTER(dbl)]
    L.fe_get_diag.argtypes = [vp, C.POINTER(_Diag)]
    L.fe_export_qdata.argtypes = [vp, vp, vp]
    L.fe_timer_read.argtypes = [vp, i32, C.POINTER(dbl), C.POINTER(i64)]
    L.fe_timer_reset.argtypes = [vp]
    L.fe_status_str.argtypes = [C.c_int]
    L.fe_status_str.restype = C.c_char_p
    L.fe_last_error.argtypes = [vp]
    L.fe_last_error.restype = C.c_char_p
    L.fe_lagrange_step.argtypes = [vp, vp, vp, vp, vp, i32, dbl, dbl, dbl, i32,
                                   C.POINTER(_StepInfo)]
    L.fe_export_l2_mass_inv.argtypes = [vp, vp]
    _lib = L
    return L


def _check(rc: int, ctx=None) -> int:
    if rc != FE_OK:
        L = lib()
        detail = L.fe_last_error(ctx).decode()
        raise FepaError(rc, f"{L.fe_status_str(rc).decode()}: {detail}")
    return rc


def _ptr(t):
    """Device pointer of a contiguous CUDA/HIP tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise FepaError(FE_EINVAL, "tensor must live on the GPU")
    if not t.is_contiguous():
        raise FepaError(FE_EINVAL, "tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class MeshDesc:
    """One mesh: host int32 map [E][(p+1)^3] (numpy), device float64 x0 [3][N] (torch)."""
    elem_nodes: object
    x0: object
    order: int
    q1d: int
    rho0: float = 1.0
    rho0_q: object = None   # device float64 [E][Q^3] initial density per point (torch), or None


@dataclass
class Opts:
    precision: int = FE_PREC_FP64
    flags: int = 0
    gamma: float = 5.0 / 3.0
    q1: float = 0.5
    q2: float = 2.0
    tune_nw_force: int = 0      # 0: tuning table / library default
    tune_nw_force_t: int = 0
    tune_nw_mass: int = 0
    tune_patch: int = 0
    tune_table: "str | None" = None   # tuning-table path (in place of FEPA_TUNE_TABLE)
    materials: "Materials | None" = None


@dataclass
class Materials:
    """Several materials: host gamma[K], rho0[K] (sequences), device eta0 [K][L2_tot] (torch)."""
    gamma: object
    rho0: object
    eta0: object


class Ctx:
    """Owns an fe_ctx_t handle (destroyed with the object)."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fe_destroy(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle


# ------------------------------------------------------------------ the ABI
def fe_pa_setup(meshes, opts: Opts | None = None, stream=None) -> Ctx:
    import numpy as np
    L = lib()
    if isinstance(meshes, MeshDesc):
        meshes = [meshes]
    descs = (_MeshDesc * len(meshes))()
    keep = []
    for k, m in enumerate(meshes):
        en = np.ascontiguousarray(m.elem_nodes, dtype=np.int32)
        keep.append(en)
        E = en.shape[0]
        descs[k] = _MeshDesc(E, m.order, m.q1d, m.x0.shape[-1], en.ctypes.data,
                             _ptr(m.x0).value, float(m.rho0),
                             None if m.rho0_q is None else _ptr(m.rho0_q).value)
    o = opts or Opts()
    co = _Opts(o.precision, o.flags, o.gamma, o.q1, o.q2, o.tune_nw_force, o.tune_nw_force_t,
               o.tune_nw_mass, o.tune_patch,
               None if o.tune_table is None else os.fsencode(o.tune_table))
    if o.materials is not None:
        mt = o.materials
        g = np.ascontiguousarray(mt.gamma, dtype=np.float64)
        r = np.ascontiguousarray(mt.rho0, dtype=np.float64)
        if g.shape != r.shape or g.ndim != 1:
            raise FepaError(FE_EINVAL, "materials: gamma and rho0 need one entry per material")
        keep += [g, r]
        cm = _Materials(len(g), g.ctypes.data, r.ctypes.data, _ptr(mt.eta0).value)
        keep.append(cm)
        co.materials = C.pointer(cm)
    h = C.c_void_p()
    _check(L.fe_pa_setup(descs, len(meshes), C.byref(co), _stream(stream), C.byref(h)))
    return Ctx(h, keep)


def fe_destroy(ctx: Ctx) -> None:
    if ctx.handle:
        lib().fe_destroy(ctx.handle)
        ctx.handle = None


def fe_query(ctx: Ctx) -> dict:
    info = _Info()
    _check(lib().fe_query(ctx.handle, C.byref(info)), ctx.handle)
    return {f: getattr(info, f) for f, _ in _Info._fields_}


def fe_mesh_offsets(ctx: Ctx):
    import numpy as np
    n = fe_query(ctx)["n_mesh"]
    a, b, c = (np.zeros(n, dtype=np.int64) for _ in range(3))
    _check(lib().fe_mesh_offsets(ctx.handle, a.ctypes.data, b.ctypes.data, c.ctypes.data),
           ctx.handle)
    return a, b, c


def fe_qdata_update(ctx: Ctx, x, v, e) -> None:
    _check(lib().fe_qdata_update(ctx.handle, _ptr(x), _ptr(v), _ptr(e)), ctx.handle)


def fe_force_mult(ctx: Ctx, e, y) -> None:
    _check(lib().fe_force_mult(ctx.handle, _ptr(e), _ptr(y)), ctx.handle)


def fe_force_mult_T(ctx: Ctx, v, z) -> None:
    _check(lib().fe_force_mult_T(ctx.handle, _ptr(v), _ptr(z)), ctx.handle)


def fe_force_mult_pair(ctx: Ctx, e, y, v, z) -> None:
    _check(lib().fe_force_mult_pair(ctx.handle, _ptr(e), _ptr(y), _ptr(v), _ptr(z)), ctx.handle)


def fe_force_mult_pair_noalloc(ctx: Ctx, e, y, v, z) -> None:
    _check(lib().fe_force_mult_pair_noalloc(ctx.handle, _ptr(e), _ptr(y), _ptr(v), _ptr(z)),
           ctx.handle)


def fe_stiffness_update(ctx: Ctx, x, kappa=None) -> None:
    _check(lib().fe_stiffness_update(ctx.handle, _ptr(x), _ptr(kappa)), ctx.handle)


def fe_stiffness_mult(ctx: Ctx, u, y) -> None:
    _check(lib().fe_stiffness_mult(ctx.handle, _ptr(u), _ptr(y)), ctx.handle)


def fe_qdata_update_mm(ctx: Ctx, x, v, e) -> None:
    _check(lib().fe_qdata_update_mm(ctx.handle, _ptr(x), _ptr(v), _ptr(e)), ctx.handle)


def fe_force_mult_T_mm(ctx: Ctx, v, z) -> None:
    _check(lib().fe_force_mult_T_mm(ctx.handle, _ptr(v), _ptr(z)), ctx.handle)


def fe_force_mult_pair_mf(ctx: Ctx, x, v, e, y, z) -> None:
    _check(lib().fe_force_mult_pair_mf(ctx.handle, _ptr(x), _ptr(v), _ptr(e), _ptr(y), _ptr(z)),
           ctx.handle)


def fe_mass_mult(ctx: Ctx, x, y) -> None:
    _check(lib().fe_mass_mult(ctx.handle, _ptr(x), _ptr(y)), ctx.handle)


def fe_mass_cg(ctx: Ctx, b, x, ess_dofs=None, rel_tol=1e-12, max_iter=1000, check=True):
    """Returns (status, iterations, true relative residual); raises unless status is OK
    (or ENOTCONV with check=False)."""
    it, rr = C.c_int32(0), C.c_double(0.0)
    n_ess = 0 if ess_dofs is None else int(ess_dofs.numel())
    rc = lib().fe_mass_cg(ctx.handle, _ptr(b), _ptr(x), _ptr(ess_dofs), n_ess, float(rel_tol),
                          int(max_iter), C.byref(it), C.byref(rr))
    if check or rc not in (FE_OK, FE_ENOTCONV):
        _check(rc, ctx.handle)
    return rc, it.value, rr.value


def fe_get_diag(ctx: Ctx) -> dict:
    d = _Diag()
    _check(lib().fe_get_diag(ctx.handle, C.byref(d)), ctx.handle)
    return {f: getattr(d, f) for f, _ in _Diag._fields_}


def fe_export_qdata(ctx: Ctx, S_out=None, mq_out=None) -> None:
    _check(lib().fe_export_qdata(ctx.handle, _ptr(S_out), _ptr(mq_out)), ctx.handle)


def fe_timer_read(ctx: Ctx, which: int):
    ms, cnt = C.c_double(0.0), C.c_int64(0)
    _check(lib().fe_timer_read(ctx.handle, which, C.byref(ms), C.byref(cnt)), ctx.handle)
    return ms.value, cnt.value


def fe_timer_reset(ctx: Ctx) -> None:
    _check(lib().fe_timer_reset(ctx.handle), ctx.handle)


def fe_status_str(status: int) -> str:
    return lib().fe_status_str(status).decode()


def fe_lagrange_step(ctx: Ctx, x, v, e, ess_dofs=None, cfl=0.5, dt_max=float("inf"),
                     cg_tol=1e-12, cg_max_iter=2000) -> dict:
    """One step of the full Lagrange phase, x, v, e updated in place; returns
    {dt, dt_est, cg_iters: [2], cg_rel_res: [2]}."""
    info = _StepInfo()
    n_ess = 0 if ess_dofs is None else int(ess_dofs.numel())
    _check(lib().fe_lagrange_step(ctx.handle, _ptr(x), _ptr(v), _ptr(e), _ptr(ess_dofs), n_ess,
                                  float(cfl), float(dt_max), float(cg_tol), int(cg_max_iter),
                                  C.byref(info)), ctx.handle)
    return {"dt": info.dt, "dt_est": info.dt_est, "cg_iters": list(info.cg_iters),
            "cg_rel_res": list(info.cg_rel_res)}


def fe_export_l2_mass_inv(ctx: Ctx, out) -> None:
    _check(lib().fe_export_l2_mass_inv(ctx.handle, _ptr(out)), ctx.handle)
