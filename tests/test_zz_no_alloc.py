"""The allocation-free force pair (fe_force_mult_pair_noalloc): the same
outputs as fe_force_mult_pair, and so as the oracle's, with the shared-node
partials held in the library's static device array. Two calls in a row, the
second on a smaller mesh, both with several patches (shared partials in use);
then a context whose partials exceed the array is rejected."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

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


def setup(torch, c, patch):
    x0 = dev(torch, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, c.p, c.Q),
                         fe.Opts(q1=c.q1, q2=c.q2, tune_patch=patch))
    x, v, e = (dev(torch, a) for a in (c.x, c.v, c.e))
    fe.fe_qdata_update(ctx, x, v, e)
    return ctx, v, e


@pytest.mark.parametrize("with_e", [False, True])
def test_noalloc_pair_matches_pair_and_oracle(torch_cuda, with_e):
    t = torch_cuda
    cases = [make_case(6, 2, 4, seed=91, permute=5, compress=0.25),   # 216 elements
             make_case(3, 3, 5, seed=92, compress=0.25)]              # 27 elements, smaller
    runs = []
    for c in cases:
        ctx, v, e = setup(t, c, patch=8)
        assert fe.fe_query(ctx)["n_elem_total"] == c.E
        ein = e if with_e else None
        yr = t.empty((3, c.N), dtype=t.float64, device="cuda")
        zr = t.empty((c.E, c.p ** 3), dtype=t.float64, device="cuda")
        fe.fe_force_mult_pair(ctx, ein, yr, v, zr)
        # outputs start as NaN: every entry must be written by the call
        y = t.full((3, c.N), float("nan"), dtype=t.float64, device="cuda")
        z = t.full((c.E, c.p ** 3), float("nan"), dtype=t.float64, device="cuda")
        runs.append((c, ctx, ein, v, yr, zr, y, z))
    # two calls in a row, the second on the smaller mesh
    for c, ctx, ein, v, yr, zr, y, z in runs:
        fe.fe_force_mult_pair_noalloc(ctx, ein, y, v, z)
    t.cuda.synchronize()
    for c, ctx, ein, v, yr, zr, y, z in runs:
        y, z, yr, zr = (a.cpu().numpy() for a in (y, z, yr, zr))
        assert np.isfinite(y).all() and np.isfinite(z).all()
        # the same kernels; only the order of the patch-local LDS sums may differ
        assert np.abs(y - yr).max() <= 1e-14 * np.abs(yr).max()
        assert np.abs(z - zr).max() <= 1e-14 * np.abs(zr).max()
        S = oracle_qdata(c)["S"]
        M, p, Q = c.mesh.elem_nodes, c.p, c.Q
        eo = c.e if with_e else None
        assert rel_cw(y, O.force_mult(M, p, Q, c.N, S, eo),
                      O.force_mult(M, p, Q, c.N, S, eo, absmode=True)) < TOL
        assert rel_cw(z, O.force_mult_T(M, p, Q, c.N, S, c.v),
                      O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)) < TOL


def test_noalloc_pair_rejects_partials_above_the_static_array(torch_cuda):
    # one element per patch: every node entry of every element is a shared
    # partial, 27 x 3 doubles per element, 54,872 elements -> 35.6 MB > 32 MiB
    t = torch_cuda
    mesh = W.cube_mesh(38, 2, 0.1, seed=93)
    x0 = dev(t, mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(mesh.elem_nodes, x0, 2, 4), fe.Opts(tune_patch=1))
    y = t.empty((3, mesh.n_nodes), dtype=t.float64, device="cuda")
    z = t.empty((mesh.n_elem, 8), dtype=t.float64, device="cuda")
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_force_mult_pair_noalloc(ctx, None, y, t.zeros_like(x0), z)
    assert ei.value.status == fe.FE_EINVAL
    assert "static scratch" in str(ei.value)
