"""Tile shapes (waves per workgroup, elements per patch) change the schedule,
never the result: every choice matches the oracle, and the tuning table named
by FEPA_TUNE_TABLE is what the library applies."""
import os

import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe

from helpers import make_case, oracle_qdata, rel_cw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("p,Q,patches", [(1, 3, (8, 64, 512)), (2, 4, (8, 64)), (3, 5, (8, 16, 64)),
                                         (3, 4, (16,)), (3, 6, (16,))])
@pytest.mark.parametrize("nw", [2, 4, 8])
def test_tile_shapes_keep_parity(torch_cuda, p, Q, patches, nw):
    # at p = 3 a request above 8 elements is cut by the 512-node tables (the
    # 4^3 mesh then has several patches: shared nodes)
    c = make_case(5 if p < 3 else 4, p, Q, seed=41, permute=1)
    qd = oracle_qdata(c)
    M, S = c.mesh.elem_nodes, qd["S"]
    y1o = O.force_mult(M, p, Q, c.N, S)
    y1a = O.force_mult(M, p, Q, c.N, S, absmode=True)
    zo = O.force_mult_T(M, p, Q, c.N, S, c.v)
    za = O.force_mult_T(M, p, Q, c.N, S, c.v, absmode=True)
    mo = O.mass_mult(M, p, Q, c.N, qd["mq"], c.v)
    ma = O.mass_mult(M, p, Q, c.N, qd["mq"], c.v, absmode=True)
    for patch in patches:
        ctx = fe.fe_pa_setup(fe.MeshDesc(M, dev(torch_cuda, c.mesh.x0), p, Q),
                             fe.Opts(tune_nw_force=nw, tune_nw_force_t=nw, tune_nw_mass=nw,
                                     tune_patch=patch))
        info = fe.fe_query(ctx)
        assert info["patch"] == patch
        x, v, e = (dev(torch_cuda, a) for a in (c.x, c.v, c.e))
        fe.fe_qdata_update(ctx, x, v, e)
        y = torch_cuda.empty((3, c.N), dtype=torch_cuda.float64, device="cuda")
        fe.fe_force_mult(ctx, None, y)
        assert rel_cw(y.cpu().numpy(), y1o, y1a) < 1e-12
        z = torch_cuda.empty((c.E, p ** 3), dtype=torch_cuda.float64, device="cuda")
        fe.fe_force_mult_T(ctx, v, z)
        assert rel_cw(z.cpu().numpy(), zo, za) < 1e-12
        fe.fe_mass_mult(ctx, v, y)
        assert rel_cw(y.cpu().numpy(), mo, ma) < 1e-12


def test_tuning_table_is_applied(torch_cuda, tmp_path):
    c = make_case(3, 2, 4, seed=42)
    table = tmp_path / "tune.txt"
    table.write_text("# p Q precision nw_force nw_force_t nw_mass patch\n2 4 0 8 2 4 8\n")
    old = os.environ.get("FEPA_TUNE_TABLE")
    os.environ["FEPA_TUNE_TABLE"] = str(table)
    try:
        ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(torch_cuda, c.mesh.x0), 2, 4))
        info = fe.fe_query(ctx)
        assert (info["nw_force"], info["nw_force_t"], info["nw_mass"], info["patch"]) == (8, 2, 4, 8)
        # explicit options override the table
        ctx2 = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(torch_cuda, c.mesh.x0), 2, 4),
                              fe.Opts(tune_nw_force=2))
        assert fe.fe_query(ctx2)["nw_force"] == 2
    finally:
        if old is None:
            del os.environ["FEPA_TUNE_TABLE"]
        else:
            os.environ["FEPA_TUNE_TABLE"] = old
