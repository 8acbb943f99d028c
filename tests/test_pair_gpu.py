"""Both force actions from one pass over S (fe_force_mult_pair): the fused
kernel must give the outputs of fe_force_mult and fe_force_mult_T, and so the
oracle's, for every (p, Q), with e and with e = 1, in FP64 and FP32, and in
batched multi-mesh contexts; in the BF16 form it reads BF16 S with FP32
contractions. The pair is also checked with several patches per mesh (nodes
shared across patches, so the shared-node partials and their gather run) and
at the full 48^3 Q2 and 64^3 Q3 workloads in the tile shapes of the built-in
table."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe

from helpers import elems_touching, make_case, oracle_qdata, rel_cw

pytestmark = pytest.mark.gpu
TOL = 1e-12
ALL_PQ = [(1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (2, 5), (3, 4), (3, 5), (3, 6), (4, 5), (4, 6),
          (4, 7)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def setup(torch, c, precision=fe.FE_PREC_FP64, flags=0, patch=0):
    x0 = dev(torch, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, c.p, c.Q),
                         fe.Opts(precision=precision, q1=c.q1, q2=c.q2, flags=flags,
                                 tune_patch=patch))
    x, v, e = (dev(torch, a) for a in (c.x, c.v, c.e))
    fe.fe_qdata_update(ctx, x, v, e)
    return ctx, v, e


@pytest.mark.parametrize("p,Q", ALL_PQ)
@pytest.mark.parametrize("with_e", [False, True])
def test_pair_matches_oracle_and_single_actions(torch_cuda, p, Q, with_e):
    t = torch_cuda
    c = make_case(3 if p <= 3 else 2, p, Q, seed=71, permute=p, compress=0.25)
    ctx, v, e = setup(t, c)
    ein = e if with_e else None
    y1, y2 = (t.empty((3, c.N), dtype=t.float64, device="cuda") for _ in range(2))
    z1, z2 = (t.empty((c.E, p ** 3), dtype=t.float64, device="cuda") for _ in range(2))
    fe.fe_force_mult_pair(ctx, ein, y1, v, z1)
    fe.fe_force_mult(ctx, ein, y2)
    fe.fe_force_mult_T(ctx, v, z2)
    y1, y2, z1, z2 = (a.cpu().numpy() for a in (y1, y2, z1, z2))
    assert np.abs(y1 - y2).max() <= 1e-14 * np.abs(y2).max()
    assert np.abs(z1 - z2).max() <= 1e-14 * np.abs(z2).max()
    S = oracle_qdata(c)["S"]
    M = c.mesh.elem_nodes
    eo = c.e if with_e else None
    assert rel_cw(y1, O.force_mult(M, p, Q, c.N, S, eo), O.force_mult(M, p, Q, c.N, S, eo, absmode=True)) < TOL
    assert rel_cw(z1, O.force_mult_T(M, p, Q, c.N, S, c.v),
                  O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)) < TOL


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5), (4, 6)])
def test_pair_fp32_equals_single_fp32_actions(torch_cuda, p, Q):
    t = torch_cuda
    c = make_case(3 if p <= 3 else 2, p, Q, seed=72)
    ctx, v, e = setup(t, c, precision=fe.FE_PREC_FP32)
    y1, y2 = (t.empty((3, c.N), dtype=t.float64, device="cuda") for _ in range(2))
    z1, z2 = (t.empty((c.E, p ** 3), dtype=t.float64, device="cuda") for _ in range(2))
    fe.fe_force_mult_pair(ctx, e, y1, v, z1)
    fe.fe_force_mult(ctx, e, y2)
    fe.fe_force_mult_T(ctx, v, z2)
    # the same FP32 arithmetic in a different summation order
    assert (y1 - y2).abs().max().item() <= 1e-6 * y2.abs().max().item()
    assert (z1 - z2).abs().max().item() <= 1e-6 * z2.abs().max().item()


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5)])
@pytest.mark.parametrize("with_e", [False, True])
def test_pair_bf16_reads_bf16_s_with_fp32_contractions(torch_cuda, p, Q, with_e):
    # The BF16 form's fused kernel reads the BF16 S and contracts it with the
    # FP32 basis table, so S's one rounding (2^-9 relative per entry) is its
    # only error beyond FP32 arithmetic: F e within 2^-9 of the term-magnitude
    # scale, and F^T v the single BF16 F^T action's up to FP32 summation order.
    t = torch_cuda
    c = make_case(3, p, Q, seed=73, permute=p, compress=0.25)
    ctx, v, e = setup(t, c, precision=fe.FE_PREC_BF16)
    ein = e if with_e else None
    y1 = t.empty((3, c.N), dtype=t.float64, device="cuda")
    z1, z2 = (t.empty((c.E, p ** 3), dtype=t.float64, device="cuda") for _ in range(2))
    fe.fe_force_mult_pair(ctx, ein, y1, v, z1)
    fe.fe_force_mult_T(ctx, v, z2)
    S = oracle_qdata(c)["S"]
    M = c.mesh.elem_nodes
    # the same FP32 products of the same BF16 S in another summation order:
    # within FP32 rounding of the sum of term magnitudes
    za = O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)
    assert (z1 - z2).abs().max().item() <= 1e-6 * np.abs(za).max()
    eo = c.e if with_e else None
    err = rel_cw(y1.cpu().numpy(), O.force_mult(M, p, Q, c.N, S, eo),
                 O.force_mult(M, p, Q, c.N, S, eo, absmode=True))
    assert err < 2.5e-3, err
    assert err > 1e-9  # and it is not an FP64 computation


@pytest.mark.parametrize("flags", [0, fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH])
def test_pair_in_multi_mesh_contexts(torch_cuda, flags):
    t = torch_cuda
    cases = [make_case(2, 1, 3, seed=74), make_case(3, 2, 4, seed=75), make_case(2, 2, 4, seed=76),
             make_case(2, 3, 5, seed=77)]
    noff = np.concatenate([[0], np.cumsum([c.N for c in cases])])
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, noff[k]:noff[k + 1]].contiguous(), c.p, c.Q)
             for k, c in enumerate(cases)]
    ctx = fe.fe_pa_setup(descs, fe.Opts(flags=flags))
    _, _, lo = fe.fe_mesh_offsets(ctx)
    L2 = fe.fe_query(ctx)["l2_size_total"]
    eh = np.zeros(L2)
    for k, c in enumerate(cases):
        eh[lo[k]:lo[k] + c.e.size] = c.e.ravel()
    x = dev(t, np.concatenate([c.x for c in cases], axis=1))
    v = dev(t, np.concatenate([c.v for c in cases], axis=1))
    e = dev(t, eh)
    fe.fe_qdata_update(ctx, x, v, e)
    y = t.empty_like(x)
    z = t.zeros(L2, dtype=t.float64, device="cuda")
    for _ in range(2):  # the second call replays the captured graph
        fe.fe_force_mult_pair(ctx, e, y, v, z)
    yh, zh = y.cpu().numpy(), z.cpu().numpy()
    for k, c in enumerate(cases):
        S = oracle_qdata(c)["S"]
        M = c.mesh.elem_nodes
        assert rel_cw(yh[:, noff[k]:noff[k + 1]], O.force_mult(M, c.p, c.Q, c.N, S, c.e),
                      O.force_mult(M, c.p, c.Q, c.N, S, c.e, absmode=True)) < TOL
        assert rel_cw(zh[lo[k]:lo[k] + c.E * c.p ** 3], O.force_mult_T(M, c.p, c.Q, c.N, S, c.v),
                      O.force_mult_T(M, c.p, c.Q, c.N, S, c.v, absmode=True)) < TOL


def test_pair_rejects_aliasing(torch_cuda):
    t = torch_cuda
    c = make_case(2, 2, 4, seed=78)
    ctx, v, e = setup(t, c)
    y = t.empty((3, c.N), dtype=t.float64, device="cuda")
    with pytest.raises(fe.FepaError):
        fe.fe_force_mult_pair(ctx, None, y, y, t.empty((c.E, 8), dtype=t.float64, device="cuda"))


@pytest.mark.parametrize("p,Q,n", [(1, 3, 6), (2, 3, 4), (2, 4, 4), (2, 5, 4), (3, 5, 3),
                                   (4, 6, 3)])
@pytest.mark.parametrize("with_e", [False, True])
def test_pair_with_several_patches(torch_cuda, p, Q, n, with_e):
    # patches of at most 8 elements (27 elements at p >= 3: a ragged last patch),
    # so nodes are shared across patches: the fused kernel leaves partials for
    # them and the gather that follows it sums them
    t = torch_cuda
    c = make_case(n, p, Q, seed=79, permute=p + 1, compress=0.25)
    ctx, v, e = setup(t, c, patch=8)
    assert fe.fe_query(ctx)["patch"] == 8
    ein = e if with_e else None
    y = t.full((3, c.N), 7.0, dtype=t.float64, device="cuda")
    z = t.full((c.E, p ** 3), 7.0, dtype=t.float64, device="cuda")
    fe.fe_force_mult_pair(ctx, ein, y, v, z)
    S = oracle_qdata(c)["S"]
    M = c.mesh.elem_nodes
    eo = c.e if with_e else None
    yh, zh = y.cpu().numpy(), z.cpu().numpy()
    assert rel_cw(yh, O.force_mult(M, p, Q, c.N, S, eo), O.force_mult(M, p, Q, c.N, S, eo, absmode=True)) < TOL
    assert rel_cw(zh, O.force_mult_T(M, p, Q, c.N, S, c.v),
                  O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)) < TOL


# the fused pair at the full workloads, in the tile shapes of the built-in table
# (the ones the benchmark times); bounds per form as in the precision tests
FULL_PAIR = [("48^3 Q2 fp64", 48, 2, 4, fe.FE_PREC_FP64, 1e-12),
             ("64^3 Q3 fp64", 64, 3, 5, fe.FE_PREC_FP64, 1e-12),
             ("64^3 Q3 fp32", 64, 3, 5, fe.FE_PREC_FP32, 1e-6),
             ("64^3 Q3 bf16", 64, 3, 5, fe.FE_PREC_BF16, 2.5e-3)]


@pytest.mark.parametrize("name,n,p,Q,prec,bound", FULL_PAIR, ids=[f[0] for f in FULL_PAIR])
def test_full_size_pair_sampled(torch_cuda, name, n, p, Q, prec, bound):
    t = torch_cuda
    c = make_case(n, p, Q, seed=0, move=0.0)
    print(f"{name}: E={c.E} N={c.N}", flush=True)
    ctx, v, e = setup(t, c, precision=prec)
    info = fe.fe_query(ctx)
    assert info["n_elem_total"] // info["patch"] > 1000   # many patches, shared nodes
    rng = np.random.default_rng(43)
    el = np.unique(np.concatenate([[0, c.E - 1], rng.integers(0, c.E, 32)])).astype(np.int32)
    nodes = np.unique(np.concatenate([[0, c.N - 1], rng.integers(0, c.N, 20)]))
    touch = elems_touching(c.mesh, nodes)
    qd = oracle_qdata(c, elems=np.union1d(el, touch).astype(np.int32))
    M = c.mesh.elem_nodes
    y = t.empty((3, c.N), dtype=t.float64, device="cuda")
    z = t.empty((c.E, p ** 3), dtype=t.float64, device="cuda")
    zo = O.force_mult_T(M, p, Q, c.N, qd["S"], c.v, elems=el)
    za = O.force_mult_T(M, p, Q, c.N, qd["S"], c.v, elems=el, absmode=True)
    for eo, ein in ((None, None), (c.e, e)):
        fe.fe_force_mult_pair(ctx, ein, y, v, z)
        yo = O.force_mult(M, p, Q, c.N, qd["S"], eo, elems=touch)
        ya = O.force_mult(M, p, Q, c.N, qd["S"], eo, elems=touch, absmode=True)
        yh, zh = y.cpu().numpy(), z.cpu().numpy()
        ey = rel_cw(yh[:, nodes], yo[:, nodes], ya[:, nodes])
        ez = rel_cw(zh[el], zo[el], za[el])
        print(f"  e={'1' if eo is None else 'e'}: F.e {ey:.2e}, F^T.v {ez:.2e}", flush=True)
        assert ey < bound and ez < bound
