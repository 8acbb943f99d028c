"""Multi-material operators on the GPU (fe_opts_t.materials,
fe_qdata_update_mm, fe_force_mult / fe_force_mult_pair on sum_k S_k, and
fe_force_mult_T_mm) against the oracle's multi-material quadrature data:
sum_k F_k 1 and every material's F_k^T v, the material and mixture masses,
for several (p, Q), with varying volume fractions, one and several patches
per mesh, and a batched two-mesh context."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

from helpers import make_case, rel_cw

pytestmark = pytest.mark.gpu
TOL = 1e-12
GAM, RHO = [5.0 / 3.0, 1.4, 3.0], [1.0, 7.8, 0.3]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def fractions(E, p, K, seed):
    # volume fractions per L2 node that sum to 1 over the materials
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.05, 1.0, (K, E, p ** 3))
    return w / w.sum(axis=0, keepdims=True)


def energies(e, K):
    return np.stack([e * (1.0 + 0.3 * k) for k in range(K)])


def run(t, cases, K, flags=0, patch=0):
    noff = np.concatenate([[0], np.cumsum([c.N for c in cases])])
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, noff[k]:noff[k + 1]].contiguous(), c.p, c.Q)
             for k, c in enumerate(cases)]
    etas = [fractions(c.E, c.p, K, 30 + k) for k, c in enumerate(cases)]
    es = [energies(c.e, K) for c in cases]
    # [K][L2_tot]: the meshes' L2 blocks in order (one order here, so no padding)
    eta = dev(t, np.concatenate([a.reshape(K, -1) for a in etas], axis=1))
    ctx = fe.fe_pa_setup(descs, fe.Opts(flags=flags, tune_patch=patch,
                                        materials=fe.Materials(GAM[:K], RHO[:K], eta)))
    x = dev(t, np.concatenate([c.x for c in cases], axis=1))
    v = dev(t, np.concatenate([c.v for c in cases], axis=1))
    e = dev(t, np.concatenate([a.reshape(K, -1) for a in es], axis=1))
    fe.fe_qdata_update_mm(ctx, x, v, e)
    N = int(noff[-1])
    L2 = e.shape[1]
    y = t.empty((3, N), dtype=t.float64, device="cuda")
    y2 = t.empty_like(y)
    zt = t.empty(L2, dtype=t.float64, device="cuda")
    z = t.empty((K, L2), dtype=t.float64, device="cuda")
    fe.fe_force_mult(ctx, None, y)
    fe.fe_force_mult_pair(ctx, None, y2, v, zt)
    fe.fe_force_mult_T_mm(ctx, v, z)
    mq = t.empty(sum(c.E * c.Q ** 3 for c in cases), dtype=t.float64, device="cuda")
    fe.fe_export_qdata(ctx, None, mq)
    out = dict(y=y.cpu().numpy(), y2=y2.cpu().numpy(), zt=zt.cpu().numpy(), z=z.cpu().numpy(),
               mq=mq.cpu().numpy())
    return out, noff, etas, es


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5), (4, 6), (2, 5)])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_multimaterial_matches_oracle(torch_cuda, p, Q, K):
    t = torch_cuda
    c = make_case(3 if p <= 3 else 2, p, Q, seed=110 + p, permute=p, compress=0.25)
    out, _, etas, es = run(t, [c], K)
    M = c.mesh.elem_nodes
    S, mqk = O.qdata_mm(M, p, Q, c.N, c.mesh.x0, c.x, c.v, es[0], etas[0], GAM[:K], RHO[:K],
                        q1=c.q1, q2=c.q2, want_mq=True)
    ref = sum(O.force_mult(M, p, Q, c.N, S[k]) for k in range(K))
    absref = sum(O.force_mult(M, p, Q, c.N, S[k], absmode=True) for k in range(K))
    assert rel_cw(out["y"], ref, absref) < TOL
    assert rel_cw(out["y2"], ref, absref) < TOL
    zsum = 0.0
    zabs = 0.0
    for k in range(K):
        zr = O.force_mult_T(M, p, Q, c.N, S[k], c.v)
        za = O.force_mult_T(M, p, Q, c.N, S[k], c.v, absmode=True)
        assert rel_cw(out["z"][k], zr, za) < TOL
        zsum, zabs = zsum + zr, zabs + za
    assert rel_cw(out["zt"], zsum, zabs) < TOL
    # the context's mass is the mixture's
    mix = mqk.sum(axis=0).ravel()
    assert np.abs(out["mq"] - mix).max() < 1e-14 * np.abs(mix).max()


def test_multimaterial_several_patches_and_batched(torch_cuda):
    t = torch_cuda
    cases = [make_case(4, 2, 4, seed=120, compress=0.2), make_case(3, 2, 4, seed=121)]
    for flags in (0, fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH):
        out, noff, etas, es = run(t, cases, 2, flags=flags, patch=8)
        loff = 0
        for k, c in enumerate(cases):
            M = c.mesh.elem_nodes
            S = O.qdata_mm(M, c.p, c.Q, c.N, c.mesh.x0, c.x, c.v, es[k], etas[k], GAM[:2], RHO[:2],
                           q1=c.q1, q2=c.q2)
            ref = O.force_mult(M, c.p, c.Q, c.N, S[0]) + O.force_mult(M, c.p, c.Q, c.N, S[1])
            absref = (O.force_mult(M, c.p, c.Q, c.N, S[0], absmode=True) +
                      O.force_mult(M, c.p, c.Q, c.N, S[1], absmode=True))
            assert rel_cw(out["y"][:, noff[k]:noff[k + 1]], ref, absref) < TOL
            L = c.E * c.p ** 3
            for m in range(2):
                zr = O.force_mult_T(M, c.p, c.Q, c.N, S[m], c.v)
                za = O.force_mult_T(M, c.p, c.Q, c.N, S[m], c.v, absmode=True)
                assert rel_cw(out["z"][m, loff:loff + L], zr, za) < TOL
            loff += L


def test_materials_rejected_where_unsupported(torch_cuda):
    t = torch_cuda
    c = make_case(2, 2, 4, seed=122)
    x0 = dev(t, c.mesh.x0)
    eta = t.ones((1, c.E * 8), dtype=t.float64, device="cuda")
    d = fe.MeshDesc(c.mesh.elem_nodes, x0, 2, 4)
    for opts, code in [(fe.Opts(precision=fe.FE_PREC_FP32, materials=fe.Materials([1.4], [1.0], eta)),
                        fe.FE_EUNSUPPORTED),
                       (fe.Opts(flags=fe.FE_OPT_STEP, materials=fe.Materials([1.4], [1.0], eta)),
                        fe.FE_EUNSUPPORTED),
                       (fe.Opts(materials=fe.Materials([0.9], [1.0], eta)), fe.FE_EINVAL)]:
        with pytest.raises(fe.FepaError) as ei:
            fe.fe_pa_setup(d, opts)
        assert ei.value.status == code
    ctx = fe.fe_pa_setup(d)
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_qdata_update_mm(ctx, x0, x0, eta)
    assert ei.value.status == fe.FE_EINVAL
