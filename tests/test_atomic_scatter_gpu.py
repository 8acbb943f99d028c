"""The atomic scatter mode (FE_OPT_ATOMIC): shared-node sums of R^T by
device-scope atomic adds instead of ordered patch partials. Every action that
scatters into the H1 space (F e, F 1, the fused pair, the allocation-free
pair, M x, the mass CG, the stiffness action, the matrix-free pair) against
the oracle at the FP64 bar, on meshes cut into several patches (shared
nodes), one and several meshes; and the CG step of a one-mesh solve, which
then reads Ap directly."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe

from helpers import make_case, oracle_qdata, rel_cw

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("p,Q,n", [(1, 3, 5), (2, 4, 4), (3, 5, 3), (2, 5, 3)])
def test_atomic_scatter_matches_oracle(torch_cuda, p, Q, n):
    t = torch_cuda
    c = make_case(n, p, Q, seed=200 + p, permute=p, compress=0.2)
    print(f"p={p} Q={Q} n={n}", flush=True)
    x0 = dev(t, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, p, Q),
                         fe.Opts(q1=c.q1, q2=c.q2, flags=fe.FE_OPT_ATOMIC | fe.FE_OPT_STIFF,
                                 tune_patch=8))
    x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
    fe.fe_qdata_update(ctx, x, v, e)
    qd = oracle_qdata(c)
    M, S = c.mesh.elem_nodes, qd["S"]
    y = t.empty_like(x)
    fe.fe_force_mult(ctx, None, y)
    assert rel_cw(y.cpu().numpy(), O.force_mult(M, p, Q, c.N, S),
                  O.force_mult(M, p, Q, c.N, S, absmode=True)) < TOL
    fe.fe_force_mult(ctx, e, y)
    assert rel_cw(y.cpu().numpy(), O.force_mult(M, p, Q, c.N, S, c.e),
                  O.force_mult(M, p, Q, c.N, S, c.e, absmode=True)) < TOL
    z = t.empty_like(e)
    zr = O.force_mult_T(M, p, Q, c.N, S, c.v)
    za = O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)
    for pair in (fe.fe_force_mult_pair, fe.fe_force_mult_pair_noalloc):
        y.fill_(7.0)  # shared nodes are zeroed by the library before the adds
        pair(ctx, None, y, v, z)
        assert rel_cw(y.cpu().numpy(), O.force_mult(M, p, Q, c.N, S),
                      O.force_mult(M, p, Q, c.N, S, absmode=True)) < TOL
        assert rel_cw(z.cpu().numpy(), zr, za) < TOL
    xr = np.random.default_rng(p).standard_normal((3, c.N))
    ym = t.empty_like(x)
    fe.fe_mass_mult(ctx, dev(t, xr), ym)
    assert rel_cw(ym.cpu().numpy(), O.mass_mult(M, p, Q, c.N, qd["mq"], xr),
                  O.mass_mult(M, p, Q, c.N, qd["mq"], xr, absmode=True)) < TOL
    # stiffness action (kappa = 1)
    fe.fe_stiffness_update(ctx, x)
    ys = t.empty_like(x)
    fe.fe_stiffness_mult(ctx, dev(t, xr), ys)
    assert rel_cw(ys.cpu().numpy(), O.stiff_mult(M, p, Q, c.N, c.x, xr),
                  O.stiff_mult(M, p, Q, c.N, c.x, xr, absmode=True)) < TOL
    # the mass CG: the one-mesh step reads the complete Ap
    b = dev(t, O.mass_mult(M, p, Q, c.N, qd["mq"], xr))
    xs = t.zeros_like(x)
    _, _, res = fe.fe_mass_cg(ctx, b, xs, rel_tol=1e-13, max_iter=2000)
    assert res < 1e-12
    assert np.abs(xs.cpu().numpy() - xr).max() < 1e-9 * np.abs(xr).max()


def test_atomic_scatter_matrix_free_pair(torch_cuda):
    t = torch_cuda
    c = make_case(4, 2, 4, seed=210, compress=0.2)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(t, c.mesh.x0), 2, 4),
                         fe.Opts(q1=c.q1, q2=c.q2, flags=fe.FE_OPT_ATOMIC, tune_patch=8))
    x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
    y = t.empty_like(x)
    z = t.empty_like(e)
    fe.fe_force_mult_pair_mf(ctx, x, v, e, y, z)
    qd = oracle_qdata(c)
    M, S = c.mesh.elem_nodes, qd["S"]
    assert rel_cw(y.cpu().numpy(), O.force_mult(M, 2, 4, c.N, S),
                  O.force_mult(M, 2, 4, c.N, S, absmode=True)) < TOL
    assert rel_cw(z.cpu().numpy(), O.force_mult_T(M, 2, 4, c.N, S, c.v),
                  O.force_mult_T(M, 2, 4, c.N, S, c.v, absmode=True)) < TOL


def test_atomic_scatter_several_meshes(torch_cuda):
    t = torch_cuda
    cases = [make_case(3, 1, 3, seed=220), make_case(4, 2, 4, seed=221, permute=2),
             make_case(2, 3, 5, seed=222)]
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    offs = np.cumsum([0] + [c.N for c in cases])
    for flags in (fe.FE_OPT_ATOMIC, fe.FE_OPT_ATOMIC | fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH):
        descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, offs[k]:offs[k + 1]].contiguous(), c.p, c.Q)
                 for k, c in enumerate(cases)]
        ctx = fe.fe_pa_setup(descs, fe.Opts(flags=flags, tune_patch=8))
        no, eo, lo = fe.fe_mesh_offsets(ctx)
        L2 = fe.fe_query(ctx)["l2_size_total"]
        eh = np.zeros(L2)
        for k, c in enumerate(cases):
            eh[lo[k]:lo[k] + c.E * c.p ** 3] = c.e.ravel()
        x = dev(t, np.concatenate([c.x for c in cases], axis=1))
        v = dev(t, np.concatenate([c.v for c in cases], axis=1))
        e = dev(t, eh)
        fe.fe_qdata_update(ctx, x, v, e)
        y = t.empty_like(x)
        fe.fe_force_mult(ctx, e, y)
        # the several-mesh CG (each mesh with its own scalars) on M x = M xr
        xr = np.random.default_rng(5).standard_normal((3, int(offs[-1])))
        b = t.empty_like(x)
        fe.fe_mass_mult(ctx, dev(t, xr), b)
        xs = t.zeros_like(x)
        fe.fe_mass_cg(ctx, b, xs, rel_tol=1e-13, max_iter=3000)
        y, bh, xh = y.cpu().numpy(), b.cpu().numpy(), xs.cpu().numpy()
        for k, c in enumerate(cases):
            qd = oracle_qdata(c)
            M = c.mesh.elem_nodes
            sl = slice(offs[k], offs[k + 1])
            assert rel_cw(y[:, sl], O.force_mult(M, c.p, c.Q, c.N, qd["S"], c.e),
                          O.force_mult(M, c.p, c.Q, c.N, qd["S"], c.e, absmode=True)) < TOL
            assert rel_cw(bh[:, sl], O.mass_mult(M, c.p, c.Q, c.N, qd["mq"], xr[:, sl]),
                          O.mass_mult(M, c.p, c.Q, c.N, qd["mq"], xr[:, sl], absmode=True)) < TOL
            assert np.abs(xh[:, sl] - xr[:, sl]).max() < 1e-9 * np.abs(xr[:, sl]).max()


@pytest.mark.parametrize("precision", [fe.FE_PREC_FP32, fe.FE_PREC_BF16])
def test_atomic_scatter_precision_forms(torch_cuda, precision):
    # the same form with the two scatter modes: they differ only in the order
    # of additions (the in-patch LDS sums, in the form's FP32, have no fixed
    # order in either mode), so by a few FP32 roundings of the summed terms
    t = torch_cuda
    c = make_case(4, 2, 4, seed=230, compress=0.2)
    outs = []
    for flags in (0, fe.FE_OPT_ATOMIC):
        ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(t, c.mesh.x0), 2, 4),
                             fe.Opts(precision=precision, flags=flags, tune_patch=8))
        x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
        fe.fe_qdata_update(ctx, x, v, e)
        y1, y2, ym = t.empty_like(x), t.empty_like(x), t.empty_like(x)
        z = t.empty_like(e)
        fe.fe_force_mult(ctx, None, y1)
        fe.fe_force_mult_pair(ctx, None, y2, v, z)
        fe.fe_mass_mult(ctx, v, ym)
        outs.append([a.cpu().numpy() for a in (y1, y2, z, ym)])
    for a, b in zip(*outs):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()
