"""Set-up options of the C ABI on the GPU: an initial density given at every
quadrature point (fe_mesh_desc_t.rho0_q, Sec. 3.3's rho |J| = rho0 |J0| with a
varying rho0) against the oracle's per-point density path, alone, in a
batched context next to a uniform-density mesh, and with FE_OPT_STEP's L2
mass; and the tuning-table path (fe_opts_t.tune_table) in place of the
environment variable."""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe

from helpers import make_case, oracle_qdata, rel_cw, rel_elem

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def density(c, seed):
    return np.random.default_rng(seed).uniform(0.5, 3.0, (c.E, c.Q ** 3))


def check_case(t, c, r0, S, mq, y, z):
    qd = O.qdata(c.mesh.elem_nodes, c.p, c.Q, c.N, c.mesh.x0, c.x, c.v, c.e, rho0=r0,
                 q1=c.q1, q2=c.q2)
    assert rel_elem(mq, qd["mq"]) < TOL
    assert rel_elem(S, qd["S"].reshape(c.E, -1)) < TOL
    M = c.mesh.elem_nodes
    assert rel_cw(y, O.force_mult(M, c.p, c.Q, c.N, qd["S"]),
                  O.force_mult(M, c.p, c.Q, c.N, qd["S"], absmode=True)) < TOL
    assert rel_cw(z, O.force_mult_T(M, c.p, c.Q, c.N, qd["S"], c.v),
                  O.force_mult_T(M, c.p, c.Q, c.N, qd["S"], c.v, absmode=True)) < TOL
    return qd


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5), (4, 6)])
def test_point_density_matches_oracle(torch_cuda, p, Q):
    t = torch_cuda
    c = make_case(3 if p <= 3 else 2, p, Q, seed=140 + p, permute=p, compress=0.2)
    r0 = density(c, 150 + p)
    x0 = dev(t, c.mesh.x0)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, p, Q, rho0_q=dev(t, r0)),
                         fe.Opts(q1=c.q1, q2=c.q2, tune_patch=8))
    x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
    fe.fe_qdata_update(ctx, x, v, e)
    Q3 = Q ** 3
    S = t.empty((c.E, 9 * Q3), dtype=t.float64, device="cuda")
    mq = t.empty((c.E, Q3), dtype=t.float64, device="cuda")
    fe.fe_export_qdata(ctx, S, mq)
    y = t.empty_like(x)
    z = t.empty_like(e)
    fe.fe_force_mult_pair(ctx, None, y, v, z)
    qd = check_case(t, c, r0, S.cpu().numpy(), mq.cpu().numpy(), y.cpu().numpy(),
                    z.cpu().numpy())
    # the mass action uses the varying density
    xr = np.random.default_rng(p).standard_normal((3, c.N))
    ym = t.empty_like(x)
    fe.fe_mass_mult(ctx, dev(t, xr), ym)
    M = c.mesh.elem_nodes
    assert rel_cw(ym.cpu().numpy(), O.mass_mult(M, p, Q, c.N, qd["mq"], xr),
                  O.mass_mult(M, p, Q, c.N, qd["mq"], xr, absmode=True)) < TOL


def test_point_density_batched_with_uniform_mesh(torch_cuda):
    t = torch_cuda
    cases = [make_case(3, 2, 4, seed=160), make_case(4, 2, 4, seed=161, permute=2)]
    r0 = density(cases[1], 162)
    x0 = dev(t, np.concatenate([c.mesh.x0 for c in cases], axis=1))
    offs = np.cumsum([0] + [c.N for c in cases])
    for flags in (0, fe.FE_OPT_BATCHED | fe.FE_OPT_GRAPH):
        descs = [fe.MeshDesc(cases[0].mesh.elem_nodes, x0[:, offs[0]:offs[1]].contiguous(), 2, 4,
                             rho0=1.7),
                 fe.MeshDesc(cases[1].mesh.elem_nodes, x0[:, offs[1]:offs[2]].contiguous(), 2, 4,
                             rho0_q=dev(t, r0))]
        ctx = fe.fe_pa_setup(descs, fe.Opts(flags=flags, tune_patch=8))
        x = dev(t, np.concatenate([c.x for c in cases], axis=1))
        v = dev(t, np.concatenate([c.v for c in cases], axis=1))
        e = dev(t, np.concatenate([c.e.ravel() for c in cases]))
        fe.fe_qdata_update(ctx, x, v, e)
        E = sum(c.E for c in cases)
        S = t.empty((E, 9 * 64), dtype=t.float64, device="cuda")
        mq = t.empty((E, 64), dtype=t.float64, device="cuda")
        fe.fe_export_qdata(ctx, S, mq)
        y = t.empty_like(x)
        z = t.empty_like(e)
        fe.fe_force_mult_pair(ctx, None, y, v, z)
        S, mq, y, z = (a.cpu().numpy() for a in (S, mq, y, z))
        e0 = 0
        for k, (c, rho) in enumerate(zip(cases, (1.7, r0))):
            sl = slice(e0, e0 + c.E)
            check_case(t, c, rho, S[sl], mq[sl], y[:, offs[k]:offs[k + 1]],
                       z[e0 * 8:(e0 + c.E) * 8])
            e0 += c.E


def test_point_density_l2_mass_of_the_step(torch_cuda):
    # FE_OPT_STEP forms M_E^-1 from m_q: with rho0_q it is the inverse of the
    # oracle's L2 mass of the varying density
    t = torch_cuda
    c = make_case(3, 2, 4, seed=170)
    r0 = density(c, 171)
    ctx = fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, dev(t, c.mesh.x0), 2, 4, rho0_q=dev(t, r0)),
                         fe.Opts(flags=fe.FE_OPT_STEP))
    out = t.empty((c.E, 8, 8), dtype=t.float64, device="cuda")
    fe.fe_export_l2_mass_inv(ctx, out)
    mq = O.qdata(c.mesh.elem_nodes, 2, 4, c.N, c.mesh.x0, c.mesh.x0, None, c.e, rho0=r0,
                 want=("mq",))["mq"]
    ME = O.l2_mass(c.mesh.elem_nodes, 2, 4, mq)
    got = out.cpu().numpy()
    for el in range(c.E):
        # the density varies sixfold: M_E is up to six times worse conditioned
        assert np.abs(got[el] @ ME[el] - np.eye(8)).max() < 1e-11


def test_point_density_rejected_values(torch_cuda):
    t = torch_cuda
    c = make_case(2, 2, 4, seed=180)
    x0 = dev(t, c.mesh.x0)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        r0 = np.ones((c.E, 64))
        r0[c.E - 1, 17] = bad
        with pytest.raises(fe.FepaError) as ei:
            fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, 2, 4, rho0_q=dev(t, r0)))
        assert ei.value.status == fe.FE_EINVAL
    eta = t.ones((1, c.E * 8), dtype=t.float64, device="cuda")
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, 2, 4, rho0_q=dev(t, np.ones((c.E, 64)))),
                       fe.Opts(materials=fe.Materials([1.4], [1.0], eta)))
    assert ei.value.status == fe.FE_EUNSUPPORTED
    # without rho0_q a non-positive uniform rho0 is still refused
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_pa_setup(fe.MeshDesc(c.mesh.elem_nodes, x0, 2, 4, rho0=0.0))
    assert ei.value.status == fe.FE_EINVAL


def test_tune_table_path(torch_cuda, tmp_path, monkeypatch):
    t = torch_cuda
    monkeypatch.delenv("FEPA_TUNE_TABLE", raising=False)
    c = make_case(4, 2, 4, seed=190)
    x0 = dev(t, c.mesh.x0)
    d = fe.MeshDesc(c.mesh.elem_nodes, x0, 2, 4)
    path = tmp_path / "tune.txt"
    path.write_text("# order q1d precision nw_force nw_force_t nw_mass patch nw_pair\n"
                    "2 4 0 4 2 4 8 4\n")
    ctx = fe.fe_pa_setup(d, fe.Opts(tune_table=str(path)))
    info = fe.fe_query(ctx)
    assert (info["nw_force"], info["nw_force_t"], info["nw_mass"], info["patch"]) == (4, 2, 4, 8)
    # the table's shapes give the oracle's results
    x, v, e = (dev(t, a) for a in (c.x, c.v, c.e))
    fe.fe_qdata_update(ctx, x, v, e)
    y = t.empty_like(x)
    z = t.empty_like(e)
    fe.fe_force_mult_pair(ctx, None, y, v, z)
    qd = oracle_qdata(c)
    M = c.mesh.elem_nodes
    assert rel_cw(y.cpu().numpy(), O.force_mult(M, 2, 4, c.N, qd["S"]),
                  O.force_mult(M, 2, 4, c.N, qd["S"], absmode=True)) < TOL
    assert rel_cw(z.cpu().numpy(), O.force_mult_T(M, 2, 4, c.N, qd["S"], c.v),
                  O.force_mult_T(M, 2, 4, c.N, qd["S"], c.v, absmode=True)) < TOL
    # the path wins over the environment variable; a missing file is an error
    other = tmp_path / "other.txt"
    other.write_text("2 4 0 2 2 8 16 2\n")
    monkeypatch.setenv("FEPA_TUNE_TABLE", str(other))
    info = fe.fe_query(fe.fe_pa_setup(d, fe.Opts(tune_table=str(path))))
    assert info["patch"] == 8
    info = fe.fe_query(fe.fe_pa_setup(d))
    assert info["patch"] == 16
    with pytest.raises(fe.FepaError) as ei:
        fe.fe_pa_setup(d, fe.Opts(tune_table=str(tmp_path / "missing.txt")))
    assert ei.value.status == fe.FE_EINVAL
