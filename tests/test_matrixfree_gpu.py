"""Fully matrix-free force pair on the GPU (fe_force_mult_pair_mf): F 1 and
F^T v of the state (x, v, e) with the quadrature data formed on the fly,
against the oracle (qdata, then the dense element force matrices) and
against the partial-assembly path (fe_qdata_update + fe_force_mult_pair), for
every (p, Q) the library builds it for, with one and several patches, in a
batched context, with its diagnostics (min detJ, stable step), and sampled
at the full 48^3 Q2 workload; unsupported pairs are refused."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

from helpers import elems_touching, make_case, oracle_qdata, rel_cw

pytestmark = pytest.mark.gpu
TOL = 1e-12
MF_PQ = [(1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (2, 5), (3, 4)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def both(t, c, patch=0):
    x0 = dev(t, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, c.p, c.Q),
                         fe.Opts(q1=c.q1, q2=c.q2, tune_patch=patch))
    x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
    y = t.full((3, c.N), float("nan"), dtype=t.float64, device="cuda")
    z = t.full((c.E, c.p ** 3), float("nan"), dtype=t.float64, device="cuda")
    fe.fe_force_mult_pair_mf(ctx, x, v, e, y, z)
    dmf = fe.fe_get_diag(ctx)
    fe.fe_qdata_update(ctx, x, v, e)
    ypa, zpa = t.empty_like(y), t.empty_like(z)
    fe.fe_force_mult_pair(ctx, None, ypa, v, zpa)
    dpa = fe.fe_get_diag(ctx)
    return [a.cpu().numpy() for a in (y, z, ypa, zpa)], dmf, dpa


@pytest.mark.parametrize("p,Q", MF_PQ)
def test_matrixfree_pair_matches_oracle_and_pa(torch_cuda, p, Q):
    t = torch_cuda
    c = make_case(3, p, Q, seed=130 + p, permute=p, compress=0.25)
    (y, z, ypa, zpa), dmf, dpa = both(t, c)
    qd = O.qdata(c.mesh.elem_nodes, p, Q, c.N, c.mesh.x0, c.x, c.v, c.e, q1=c.q1, q2=c.q2,
                 want=("S", "detJ", "dt"))
    S, M = qd["S"], c.mesh.elem_nodes
    assert rel_cw(y, O.force_mult(M, p, Q, c.N, S), O.force_mult(M, p, Q, c.N, S, absmode=True)) < TOL
    assert rel_cw(z, O.force_mult_T(M, p, Q, c.N, S, c.v),
                  O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)) < TOL
    assert np.abs(y - ypa).max() <= 1e-13 * np.abs(ypa).max()
    assert np.abs(z - zpa).max() <= 1e-13 * np.abs(zpa).max()
    assert abs(dmf["min_detj"] - qd["detJ"].min()) <= 1e-14 * qd["detJ"].max()
    assert abs(dmf["dt_est"] - qd["dt"].min()) <= 1e-13 * qd["dt"].min()
    assert dmf["nonfinite"] == 0


@pytest.mark.parametrize("p,Q,n", [(1, 3, 6), (2, 4, 5), (3, 4, 4)])
def test_matrixfree_pair_several_patches(torch_cuda, p, Q, n):
    t = torch_cuda
    c = make_case(n, p, Q, seed=140 + p)
    (y, z, ypa, zpa), _, _ = both(t, c, patch=8)
    S, M = oracle_qdata(c)["S"], c.mesh.elem_nodes
    assert rel_cw(y, O.force_mult(M, p, Q, c.N, S), O.force_mult(M, p, Q, c.N, S, absmode=True)) < TOL
    assert rel_cw(z, O.force_mult_T(M, p, Q, c.N, S, c.v),
                  O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)) < TOL


def test_matrixfree_pair_batched(torch_cuda):
    t = torch_cuda
    cases = [make_case(3, 2, 4, seed=150), make_case(2, 1, 3, seed=151), make_case(2, 2, 4, seed=152)]
    noff = np.concatenate([[0], np.cumsum([c.N for c in cases])])
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, noff[k]:noff[k + 1]].contiguous(), c.p, c.Q)
             for k, c in enumerate(cases)]
    ctx = fe.fe_pa_setup(descs, fe.Opts(flags=fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH, tune_patch=8))
    _, _, loff = fe.fe_mesh_offsets(ctx)
    L2 = fe.fe_query(ctx)["l2_size_total"]
    e = np.zeros(L2)
    for k, c in enumerate(cases):
        e[loff[k]:loff[k] + c.e.size] = c.e.ravel()
    x = dev(t, np.concatenate([c.x for c in cases], axis=1))
    v = dev(t, np.concatenate([c.v for c in cases], axis=1))
    y = t.empty((3, int(noff[-1])), dtype=t.float64, device="cuda")
    z = t.zeros(L2, dtype=t.float64, device="cuda")
    fe.fe_force_mult_pair_mf(ctx, x, v, dev(t, e), y, z)
    y, z = y.cpu().numpy(), z.cpu().numpy()
    for k, c in enumerate(cases):
        S, M = oracle_qdata(c)["S"], c.mesh.elem_nodes
        assert rel_cw(y[:, noff[k]:noff[k + 1]], O.force_mult(M, c.p, c.Q, c.N, S),
                      O.force_mult(M, c.p, c.Q, c.N, S, absmode=True)) < TOL
        zk = z[loff[k]:loff[k] + c.e.size].reshape(c.E, -1)
        assert rel_cw(zk, O.force_mult_T(M, c.p, c.Q, c.N, S, c.v),
                      O.force_mult_T(M, c.p, c.Q, c.N, S, c.v, absmode=True)) < TOL


def test_matrixfree_pair_refuses_unbuilt_pairs(torch_cuda):
    t = torch_cuda
    c = make_case(2, 3, 5, seed=153)
    x0 = dev(t, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, 3, 5))
    y = t.empty((3, c.N), dtype=t.float64, device="cuda")
    z = t.empty((c.E, 27), dtype=t.float64, device="cuda")
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_force_mult_pair_mf(ctx, x0, x0.clone(), dev(t, c.e), y, z)
    assert ei.value.status == fe.FE_EUNSUPPORTED


def test_matrixfree_pair_full_size_c2_sampled(torch_cuda):
    t = torch_cuda
    n, p, Q = 48, 2, 4
    mesh = W.cube_mesh(n, p, W.default_amp(p), seed=0)
    v, e = W.taylor_green_fields(mesh)
    x = mesh.x0 + 0.05 / n * v
    x0 = dev(t, mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(mesh.elem_nodes, x0, p, Q))
    y = t.empty((3, mesh.n_nodes), dtype=t.float64, device="cuda")
    z = t.empty((mesh.n_elem, p ** 3), dtype=t.float64, device="cuda")
    fe.fe_force_mult_pair_mf(ctx, dev(t, x), dev(t, v), dev(t, e), y, z)
    y, z = y.cpu().numpy(), z.cpu().numpy()
    rng = np.random.default_rng(12)
    nodes = np.unique(np.concatenate([rng.choice(mesh.n_nodes, 60, replace=False),
                                      mesh.elem_nodes[rng.choice(mesh.n_elem, 4)].ravel()]))
    el = elems_touching(mesh, nodes)
    M = mesh.elem_nodes
    qd = O.qdata(M, p, Q, mesh.n_nodes, mesh.x0, x, v, e, elems=el, want=("S",))
    ref = O.force_mult(M, p, Q, mesh.n_nodes, qd["S"], elems=el)
    absref = O.force_mult(M, p, Q, mesh.n_nodes, qd["S"], elems=el, absmode=True)
    assert rel_cw(y[:, nodes], ref[:, nodes], absref[:, nodes]) < TOL
    zr = O.force_mult_T(M, p, Q, mesh.n_nodes, qd["S"], v, elems=el)
    za = O.force_mult_T(M, p, Q, mesh.n_nodes, qd["S"], v, elems=el, absmode=True)
    assert rel_cw(z[el], zr[el], za[el]) < TOL
