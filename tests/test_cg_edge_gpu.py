"""Edge cases of the mass CG on the GPU: a zero right side gives the exact
solution x = 0 with no iteration whatever the first guess, in a one-mesh
context and per mesh in a batched one (the other mesh still solved to the
oracle's solution); and solves on one context that need more, then fewer,
iterations than the one before (the first poll of the device state goes out
where the last solve ended) give the same counts and answers as the first."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

from helpers import make_case, oracle_qdata

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_zero_rhs_one_mesh(torch_cuda):
    t = torch_cuda
    c = make_case(3, 2, 4, seed=160)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(t, c.mesh.x0), 2, 4))
    x = dev(t, np.random.default_rng(1).standard_normal((3, c.N)))
    b = t.zeros_like(x)
    rc, it, rr = fe.fe_mass_cg(ctx, b, x, dev(t, W.boundary_normal_dofs(c.mesh)), rel_tol=1e-12)
    assert rc == 0 and it == 0 and rr == 0.0
    assert x.abs().max().item() == 0.0


def test_zero_rhs_on_one_mesh_of_a_batch(torch_cuda):
    t = torch_cuda
    cases = [make_case(3, 2, 4, seed=161), make_case(2, 3, 5, seed=162)]
    noff = np.concatenate([[0], np.cumsum([c.N for c in cases])])
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    descs = [fe.MeshDesc(c.mesh.elem_nodes, x0[:, noff[k]:noff[k + 1]].contiguous(), c.p, c.Q)
             for k, c in enumerate(cases)]
    ctx = fe.fe_pa_setup(descs, fe.Opts(flags=fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH))
    N = int(noff[-1])
    rng = np.random.default_rng(2)
    b = np.zeros((3, N))
    b[:, noff[1]:] = rng.standard_normal((3, cases[1].N))
    x = dev(t, rng.standard_normal((3, N)))
    rc, it, rr = fe.fe_mass_cg(ctx, dev(t, b), x, None, rel_tol=1e-12, max_iter=3000)
    assert rc == 0 and rr < 2e-12
    xg = x.cpu().numpy()
    assert np.abs(xg[:, :noff[1]]).max() == 0.0
    c = cases[1]
    mq = O.qdata(c.mesh.elem_nodes, c.p, c.Q, c.N, c.mesh.x0, c.mesh.x0, None, None, want=("mq",))["mq"]
    xo, _, _, ok = O.mass_cg(c.mesh.elem_nodes, c.p, c.Q, c.N, mq, b[:, noff[1]:], rel_tol=1e-13,
                             max_iter=5000)
    assert ok
    assert np.linalg.norm(xg[:, noff[1]:] - xo) <= 1e-9 * np.linalg.norm(xo)


@pytest.mark.parametrize("flags", [0, fe.FE_OPT_GRAPH])
def test_solves_longer_then_shorter_than_the_last(torch_cuda, flags):
    t = torch_cuda
    c = make_case(4, 2, 4, seed=163)
    M = c.mesh.elem_nodes
    ctx = fe.fe_pa_setup(fe.MeshDesc(M, dev(t, c.mesh.x0), 2, 4), fe.Opts(flags=flags))
    mq = O.qdata(M, 2, 4, c.N, c.mesh.x0, c.mesh.x0, None, None, want=("mq",))["mq"]
    xr = np.random.default_rng(3).standard_normal((3, c.N))
    b = dev(t, O.mass_mult(M, 2, 4, c.N, mq, xr))
    runs = {}
    # loose, tight (past the loose count), loose (far short of the tight count), tight
    for tol in (1e-4, 1e-12, 1e-4, 1e-12):
        x = t.zeros_like(b)
        rc, it, rr = fe.fe_mass_cg(ctx, b, x, rel_tol=tol, max_iter=2000)
        print(f"flags={flags} tol={tol} iters={it} res={rr:.3e}", flush=True)
        assert rc == 0 and rr < 2 * tol
        runs.setdefault(tol, []).append((it, x.cpu().numpy()))
    assert runs[1e-4][0][0] < runs[1e-12][0][0]
    for (i1, x1), (i2, x2) in runs.values():
        # the patch sums have no fixed order, so a count may move by one
        assert abs(i1 - i2) <= 1
        assert np.abs(x1 - x2).max() <= 1e-3 * np.abs(x1).max()
    assert np.abs(runs[1e-12][1][1] - xr).max() < 1e-8 * np.abs(xr).max()
