"""The full Lagrange step on the GPU (fe_lagrange_step): the semi-discrete
system of Sec. 3.3 advanced by the two-stage scheme, checked against the
oracle's step, and at the full 48^3 Q2 workload against properties the
oracle evaluates (total energy, the stable step, the walls).

Tolerances: the step contains two CG solves to a relative residual tol, so
the acceleration, and with it every increment of the state, carries a
relative error of about cond(M_v) * tol (cond ~ 1e2 at these meshes); the
increments are compared at 1e-9 of their size with tol = 1e-13 on the GPU
and 1e-14 in the oracle. The element inverses of M_E have no solve in them
and are checked at 1e-12."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

from helpers import make_case

pytestmark = pytest.mark.gpu
ALL_PQ = [(1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (2, 5), (3, 4), (3, 5), (3, 6), (4, 5), (4, 6),
          (4, 7)]
INC_TOL = 1e-9


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def walled_case(n, p, Q=None, seed=0, move=0.0):
    c = make_case(n, p, Q, seed=seed, move=move)
    ess = W.boundary_normal_dofs(c.mesh)
    c.v.ravel()[ess] = 0.0
    return c, ess


def gpu_ctx(torch, c, flags=fe.FE_OPT_STEP, patch=0):
    x0 = dev(torch, c.mesh.x0)
    return fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, c.p, c.Q),
                          fe.Opts(q1=c.q1, q2=c.q2, flags=flags, tune_patch=patch))


def close_increment(got, ref, base, tol=INC_TOL):
    d_got, d_ref = np.asarray(got) - base, np.asarray(ref) - base
    scale = np.abs(d_ref).max()
    return float(np.abs(d_got - d_ref).max() / (scale if scale > 0 else 1.0)) < tol


@pytest.mark.parametrize("p,Q", ALL_PQ)
def test_l2_mass_inverse(torch_cuda, p, Q):
    c = make_case(2 if p == 4 else 3, p, Q, seed=41, permute=p)
    ctx = gpu_ctx(torch_cuda, c)
    Dl3 = p ** 3
    out = torch_cuda.empty((c.E, Dl3, Dl3), dtype=torch_cuda.float64, device="cuda")
    fe.fe_export_l2_mass_inv(ctx, out)
    mq = O.qdata(c.mesh.elem_nodes, p, Q, c.N, c.mesh.x0, c.mesh.x0, None, None, want=("mq",))["mq"]
    ME = O.l2_mass(c.mesh.elem_nodes, p, Q, mq)
    prod = np.einsum("ejk,ekl->ejl", out.cpu().numpy(), ME)
    assert np.abs(prod - np.eye(Dl3)[None]).max() < 1e-12


@pytest.mark.parametrize("p,Q,n", [(1, 3, 4), (2, 4, 3), (2, 3, 3), (3, 5, 2), (4, 6, 2)])
def test_step_matches_oracle(torch_cuda, p, Q, n):
    t = torch_cuda
    c, ess = walled_case(n, p, Q, seed=42)
    ctx = gpu_ctx(t, c)
    x, v, e = (dev(t, a) for a in (c.mesh.x0, c.v, c.e))
    info = fe.fe_lagrange_step(ctx, x, v, e, dev(t, ess), cfl=0.5, cg_tol=1e-13)
    M = c.mesh.elem_nodes
    dtq = O.qdata(M, p, Q, c.N, c.mesh.x0, c.mesh.x0, c.v, c.e, q1=c.q1, q2=c.q2,
                  want=("dt",))["dt"].min()
    assert abs(info["dt_est"] - dtq) <= 1e-13 * dtq
    assert abs(info["dt"] - 0.5 * dtq) <= 1e-13 * dtq
    xo, vo, eo, dto = O.lagrange_step(M, p, Q, c.N, c.mesh.x0, c.mesh.x0, c.v, c.e, ess=ess,
                                      cfl=1e9, dt_max=info["dt"], q1=c.q1, q2=c.q2)
    assert dto == info["dt"]
    xg, vg, eg = (a.cpu().numpy() for a in (x, v, e))
    print(f"p={p} Q={Q}: dt {info['dt']:.4e}, CG {info['cg_iters']}", flush=True)
    assert close_increment(xg, xo, c.mesh.x0)
    assert close_increment(vg, vo, c.v)
    assert close_increment(eg, eo, c.e)
    assert np.all(vg.ravel()[ess] == 0.0)


def test_several_steps_and_energy(torch_cuda):
    # five steps of the 4^3 Q2 workload: the state follows the oracle's and the
    # total energy (evaluated by the oracle from the GPU state) stays constant
    t = torch_cuda
    p, Q = 2, 4
    c, ess = walled_case(4, p, Q, seed=0)
    M, N = c.mesh.elem_nodes, c.N
    ctx = gpu_ctx(t, c)
    x, v, e = (dev(t, a) for a in (c.mesh.x0, c.v, c.e))
    xo, vo, eo = c.mesh.x0.copy(), c.v.copy(), c.e.copy()
    mq = O.qdata(M, p, Q, N, c.mesh.x0, c.mesh.x0, None, None, want=("mq",))["mq"]
    k0, i0 = O.total_energy(M, p, Q, N, mq, c.v, c.e)
    for step in range(5):
        info = fe.fe_lagrange_step(ctx, x, v, e, dev(t, ess), cfl=0.5, cg_tol=1e-13)
        xo, vo, eo, _ = O.lagrange_step(M, p, Q, N, c.mesh.x0, xo, vo, eo, ess=ess, cfl=1e9,
                                        dt_max=info["dt"], q1=c.q1, q2=c.q2)
    xg, vg, eg = (a.cpu().numpy() for a in (x, v, e))
    assert close_increment(xg, xo, c.mesh.x0, 1e-8)
    assert close_increment(vg, vo, c.v, 1e-8)
    assert close_increment(eg, eo, c.e, 1e-8)
    k1, i1 = O.total_energy(M, p, Q, N, mq, vg, eg)
    assert abs(k1 - k0) > 1e-4 * k0
    assert abs((k1 + i1) - (k0 + i0)) < 1e-12 * (k0 + i0)


def test_still_gas_and_dt_max(torch_cuda):
    # v = 0 and uniform e between walls: nothing moves; dt_max caps the step
    t = torch_cuda
    p, Q = 2, 4
    mesh = W.cube_mesh(3, p, 0.1, seed=43)
    x0 = dev(t, mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(mesh.elem_nodes, x0, p, Q), fe.Opts(flags=fe.FE_OPT_STEP))
    ess = dev(t, W.boundary_normal_dofs(mesh))
    x, v = x0.clone(), t.zeros_like(x0)
    e = t.full((mesh.n_elem, p ** 3), 3.0, dtype=t.float64, device="cuda")
    info = fe.fe_lagrange_step(ctx, x, v, e, ess, cfl=0.5, dt_max=1e-4)
    assert info["dt"] == 1e-4
    p0 = (5.0 / 3.0 - 1.0) * 3.0
    vmax = 1e-12 * p0 * 1e-4 * 3        # roundoff on the scale p0 dt / h
    assert v.abs().max().item() < vmax
    assert (e - 3.0).abs().max().item() < 1e-13
    assert (x - x0).abs().max().item() < vmax * 1e-4
    # no pressure and no motion: no finite step unless dt_max gives one (v
    # exactly 0: the roundoff motion left by the step above would give the
    # quadratic viscosity a tiny finite speed)
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_lagrange_step(ctx, x, t.zeros_like(v), t.zeros_like(e), ess, cfl=0.5)
    assert ei.value.status == fe.FE_EINVAL


def test_step_needs_the_option(torch_cuda):
    t = torch_cuda
    c, ess = walled_case(2, 2, 4)
    ctx = gpu_ctx(t, c, flags=0)
    x, v, e = (dev(t, a) for a in (c.mesh.x0, c.v, c.e))
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_lagrange_step(ctx, x, v, e, dev(t, ess))
    assert ei.value.status == fe.FE_EINVAL


def test_step_several_patches_and_meshes(torch_cuda):
    # a two-mesh batched context (one dt for both) with 8-element patches
    t = torch_cuda
    cases = [walled_case(4, 2, 4, seed=44), walled_case(3, 3, 5, seed=45)]
    noff = np.concatenate([[0], np.cumsum([c.N for c, _ in cases])])
    x0 = dev(t, np.concatenate([c.mesh.x0 for c, _ in cases], axis=1))
    descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, noff[k]:noff[k + 1]].contiguous(), c.p, c.Q)
             for k, (c, _) in enumerate(cases)]
    ctx = fe.fe_pa_setup(descs, fe.Opts(flags=fe.FE_OPT_STEP | fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH,
                                        tune_patch=8))
    _, _, lo = fe.fe_mesh_offsets(ctx)
    L2 = fe.fe_query(ctx)["l2_size_total"]
    eh = np.zeros(L2)
    for k, (c, _) in enumerate(cases):
        eh[lo[k]:lo[k] + c.e.size] = c.e.ravel()
    ess = np.concatenate([(ess_k // c.N) * noff[-1] + noff[k] + ess_k % c.N
                          for k, (c, ess_k) in enumerate(cases)]).astype(np.int32)
    x = x0.clone()
    v = dev(t, np.concatenate([c.v for c, _ in cases], axis=1))
    e = dev(t, eh)
    info = fe.fe_lagrange_step(ctx, x, v, e, dev(t, ess), cfl=0.5, cg_tol=1e-13)
    dts = [O.qdata(c.mesh.elem_nodes, c.p, c.Q, c.N, c.mesh.x0, c.mesh.x0, c.v, c.e,
                   want=("dt",))["dt"].min() for c, _ in cases]
    assert abs(info["dt"] - 0.5 * min(dts)) <= 1e-13 * min(dts)
    xg, vg, eg = (a.cpu().numpy() for a in (x, v, e))
    for k, (c, ess_k) in enumerate(cases):
        xo, vo, eo, _ = O.lagrange_step(c.mesh.elem_nodes, c.p, c.Q, c.N, c.mesh.x0, c.mesh.x0, c.v,
                                        c.e, ess=ess_k, cfl=1e9, dt_max=info["dt"])
        sl = slice(noff[k], noff[k + 1])
        assert close_increment(xg[:, sl], xo, c.mesh.x0)
        assert close_increment(vg[:, sl], vo, c.v)
        assert close_increment(eg[lo[k]:lo[k] + c.e.size].reshape(c.e.shape), eo, c.e)


def test_full_size_step_c2(torch_cuda):
    """One step of the 48^3 Q2 workload: the stable step the oracle computes on
    every point, the walls, and the total energy (oracle functionals of the
    GPU state) conserved to the CG tolerance."""
    t = torch_cuda
    p, Q = 2, 4
    c, ess = walled_case(48, p, Q, seed=0)
    M, N = c.mesh.elem_nodes, c.N
    ctx = gpu_ctx(t, c)
    x, v, e = (dev(t, a) for a in (c.mesh.x0, c.v, c.e))
    info = fe.fe_lagrange_step(ctx, x, v, e, dev(t, ess), cfl=0.5, cg_tol=1e-12)
    print(f"C2 step: dt {info['dt']:.4e}, CG {info['cg_iters']} res {info['cg_rel_res']}", flush=True)
    qd = O.qdata(M, p, Q, N, c.mesh.x0, c.mesh.x0, c.v, c.e, q1=c.q1, q2=c.q2, want=("dt", "mq"))
    assert abs(info["dt_est"] - qd["dt"].min()) <= 1e-13 * qd["dt"].min()
    vg, eg = v.cpu().numpy(), e.cpu().numpy()
    assert np.all(vg.ravel()[ess] == 0.0)
    k0, i0 = O.total_energy(M, p, Q, N, qd["mq"], c.v, c.e)
    k1, i1 = O.total_energy(M, p, Q, N, qd["mq"], vg, eg)
    assert abs(k1 - k0) > 1e-6 * k0
    assert abs((k1 + i1) - (k0 + i0)) < 1e-11 * (k0 + i0)
