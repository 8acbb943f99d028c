"""Batching form on the GPU: many meshes of uneven size and order in one context.

With FE_OPT_BATCHED every (order, Q) class of meshes is one launch unit over
the concatenated patch plans of its meshes; with FE_OPT_GRAPH each action (and
each group of CG iterations) is replayed from a captured hipGraph in which the
unit launches are parallel branches. Every output must match the oracle mesh by
mesh, and the per-mesh launches of the plain path up to summation order.
"""
import numpy as np
import pytest

import oracle as O
import paper_2112_07075_amd as fe
from paper_2112_07075_amd import workload as W

from helpers import make_case, oracle_qdata, rel_cw

pytestmark = pytest.mark.gpu
TOL = 1e-12
B, G = fe.FE_OPT_BATCHED, fe.FE_OPT_GRAPH
FLAGS = [0, B, G, B | G]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# (n, p, Q, seed): three classes share (p, p+2), one mesh has Q = p+1, sizes ragged
SPECS = [(2, 1, 3, 41), (3, 2, 4, 42), (2, 3, 5, 43), (3, 1, 3, 44), (2, 2, 4, 45),
         (1, 4, 6, 46), (2, 2, 3, 47), (1, 1, 3, 48)]


def mixed_cases():
    return [make_case(n, p, Q, seed=s, permute=s, compress=0.2) for n, p, Q, s in SPECS]


class Multi:
    """One context over several meshes; inputs laid out by the library's offsets."""

    def __init__(self, torch, meshes, qs, flags, fields=None):
        self.torch = torch
        N = [m.n_nodes for m in meshes]
        self.noff = np.concatenate([[0], np.cumsum(N)]).astype(np.int64)
        x0 = dev(torch, np.concatenate([m.x0 for m in meshes], axis=1))
        self.descs = [fe.MeshDesc(m.elem_nodes, x0[:, self.noff[k]:self.noff[k + 1]].contiguous(),
                                  m.p, qs[k]) for k, m in enumerate(meshes)]
        self.ctx = fe.fe_pa_setup(self.descs, fe.Opts(flags=flags))
        no, self.eoff, self.loff = fe.fe_mesh_offsets(self.ctx)
        assert list(no) == list(self.noff[:-1])
        self.L2 = fe.fe_query(self.ctx)["l2_size_total"]
        self.meshes = meshes
        self.Ntot = int(self.noff[-1])

    def h1(self, parts):
        return dev(self.torch, np.concatenate(parts, axis=1))

    def l2(self, parts):
        a = np.zeros(self.L2)
        for k, p in enumerate(parts):
            a[self.loff[k]:self.loff[k] + p.size] = p.ravel()
        return dev(self.torch, a)

    def l2_slice(self, a, k):
        m = self.meshes[k]
        return a[self.loff[k]:self.loff[k] + m.n_elem * m.p ** 3]

    def h1_slice(self, a, k):
        return a[:, self.noff[k]:self.noff[k + 1]]

    def actions(self, x, v, e, xr):
        t = self.torch
        fe.fe_qdata_update(self.ctx, x, v, e)
        y = t.empty((3, self.Ntot), dtype=t.float64, device="cuda")
        out = {}
        fe.fe_force_mult(self.ctx, None, y)
        out["F1"] = y.cpu().numpy()
        fe.fe_force_mult(self.ctx, e, y)
        out["Fe"] = y.cpu().numpy()
        z = t.zeros(self.L2, dtype=t.float64, device="cuda")
        fe.fe_force_mult_T(self.ctx, v, z)
        out["FTv"] = z.cpu().numpy()
        fe.fe_mass_mult(self.ctx, xr, y)
        out["Mx"] = y.cpu().numpy()
        return out


def run_mixed(torch, flags):
    cases = mixed_cases()
    g = Multi(torch, [c.mesh for c in cases], [c.Q for c in cases], flags)
    xr = np.random.default_rng(5).standard_normal((3, g.Ntot))
    out = g.actions(g.h1([c.x for c in cases]), g.h1([c.v for c in cases]),
                    g.l2([c.e for c in cases]), dev(torch, xr))
    return cases, g, out, xr


@pytest.mark.parametrize("flags", FLAGS)
def test_mixed_batch_matches_oracle(torch_cuda, flags):
    cases, g, out, xr = run_mixed(torch_cuda, flags)
    for k, c in enumerate(cases):
        qd = oracle_qdata(c)
        M, S = c.mesh.elem_nodes, qd["S"]
        ref = {
            "F1": (O.force_mult(M, c.p, c.Q, c.N, S), O.force_mult(M, c.p, c.Q, c.N, S, absmode=True)),
            "Fe": (O.force_mult(M, c.p, c.Q, c.N, S, c.e),
                   O.force_mult(M, c.p, c.Q, c.N, S, c.e, absmode=True)),
            "Mx": (O.mass_mult(M, c.p, c.Q, c.N, qd["mq"], g.h1_slice(xr, k)),
                   O.mass_mult(M, c.p, c.Q, c.N, qd["mq"], g.h1_slice(xr, k), absmode=True)),
        }
        for name, (r, a) in ref.items():
            err = rel_cw(g.h1_slice(out[name], k), r, a)
            assert err < TOL, (k, name, err)
        zo = O.force_mult_T(M, c.p, c.Q, c.N, S, c.v)
        za = O.force_mult_T(M, c.p, c.Q, c.N, S, c.v, absmode=True)
        err = rel_cw(g.l2_slice(out["FTv"], k), zo, za)
        assert err < TOL, (k, "FTv", err)
    # padding between L2 blocks is never written
    covered = np.zeros(g.L2, dtype=bool)
    for k, c in enumerate(cases):
        covered[g.loff[k]:g.loff[k] + c.E * c.p ** 3] = True
    assert np.all(out["FTv"][~covered] == 0.0)


@pytest.mark.parametrize("flags", [B, G, B | G])
def test_mixed_batch_equals_per_mesh_launches(torch_cuda, flags):
    _, _, ref, _ = run_mixed(torch_cuda, 0)
    _, _, got, _ = run_mixed(torch_cuda, flags)
    for name in ref:
        scale = np.abs(ref[name]).max()
        assert np.abs(got[name] - ref[name]).max() <= 1e-14 * scale, name


def close(a, b):
    """Equal up to summation order (the patch kernels add element contributions in
    LDS with atomics, so the order of equal-rank terms varies between runs)."""
    return (a - b).abs().max().item() <= 1e-14 * b.abs().max().item()


def test_graph_replays_follow_changing_inputs(torch_cuda):
    """Replays of one captured graph (same pointers, new contents, eager work and
    synchronisation in between) reproduce the eager launches of the same plan;
    the inputs change by 1e-2 between replays, far above the tolerance."""
    t = torch_cuda
    cases = mixed_cases()
    meshes, qs = [c.mesh for c in cases], [c.Q for c in cases]
    ge = Multi(t, meshes, qs, B)
    gg = Multi(t, meshes, qs, B | G)
    x = ge.h1([c.x for c in cases])
    v = ge.h1([c.v for c in cases])
    e = ge.l2([c.e for c in cases])
    y1, y2 = (t.empty_like(x) for _ in range(2))
    z1, z2 = (t.zeros(ge.L2, dtype=t.float64, device="cuda") for _ in range(2))
    gen = t.Generator(device="cuda").manual_seed(3)
    for rep in range(4):
        v.add_(0.01 * t.randn(v.shape, generator=gen, device="cuda", dtype=t.float64))
        t.cuda.synchronize()
        for g, y, z in ((ge, y1, z1), (gg, y2, z2)):
            fe.fe_qdata_update(g.ctx, x, v, e)
            fe.fe_force_mult(g.ctx, e, y)
            fe.fe_force_mult_T(g.ctx, v, z)
        t.cuda.synchronize()
        assert close(y2, y1), rep
        assert close(z2, z1), rep
        fe.fe_mass_mult(ge.ctx, v, y1)
        fe.fe_mass_mult(gg.ctx, v, y2)
        t.cuda.synchronize()
        assert close(y2, y1), rep


@pytest.mark.parametrize("flags", FLAGS)
@pytest.mark.parametrize("ess", [False, True])
def test_mixed_batch_cg(torch_cuda, flags, ess):
    t = torch_cuda
    cases = mixed_cases()
    g = Multi(t, [c.mesh for c in cases], [c.Q for c in cases], flags)
    rng = np.random.default_rng(8)
    xs, bs, ess_all = [], [], []
    for k, c in enumerate(cases):
        xk = rng.standard_normal((3, c.N))
        if ess:
            idx = W.boundary_normal_dofs(c.mesh)
            xk.ravel()[idx] = 0.0
            comp, node = idx // c.N, idx % c.N
            ess_all.append(comp * g.Ntot + g.noff[k] + node)
        xs.append(xk)
        bs.append(O.mass_mult(c.mesh.elem_nodes, c.p, c.Q, c.N, oracle_qdata(c)["mq"], xk))
    xs = np.concatenate(xs, axis=1)
    ess_t = dev(t, np.concatenate(ess_all).astype(np.int32)) if ess else None
    b = g.h1(bs)
    xg = t.zeros((3, g.Ntot), dtype=t.float64, device="cuda")
    for rep in range(2):  # the second solve replays the captured CG graphs
        xg.zero_()
        rc, it, rr = fe.fe_mass_cg(g.ctx, b, xg, ess_t, rel_tol=1e-12)
        xh = xg.cpu().numpy()
        assert rc == fe.FE_OK and rr <= 1e-12, (rep, rr)
        assert np.linalg.norm(xh - xs) < 1e-9 * np.linalg.norm(xs), rep


def test_batch_workload_full_size_batched_vs_per_mesh(torch_cuda):
    """The 256-mesh uneven batch (4^3..24^3 elements, p 1..4, Q = p+2): batched
    graph replays against per-mesh launches, and the two smallest meshes of each
    order against the oracle."""
    t = torch_cuda
    items = W.batch_meshes(256)
    meshes, qs = [b.mesh for b in items], [b.q1d for b in items]
    fields = [W.taylor_green_fields(m) for m in meshes]
    res = {}
    for flags in (0, B | G):
        g = Multi(t, meshes, qs, flags)
        x = g.h1([m.x0 for m in meshes])
        v = g.h1([f[0] for f in fields])
        e = g.l2([f[1] for f in fields])
        fe.fe_qdata_update(g.ctx, x, v, e)
        y = t.empty_like(x)
        fe.fe_force_mult(g.ctx, None, y)
        z = t.zeros(g.L2, dtype=t.float64, device="cuda")
        fe.fe_force_mult_T(g.ctx, v, z)
        res[flags] = (y.cpu().numpy(), z.cpu().numpy())
        del g, x, v, e, y, z
        t.cuda.empty_cache()
    (y0, z0), (y1, z1) = res[0], res[B | G]
    assert np.abs(y1 - y0).max() <= 1e-14 * np.abs(y0).max()
    assert np.abs(z1 - z0).max() <= 1e-14 * np.abs(z0).max()
    noff = np.concatenate([[0], np.cumsum([m.n_nodes for m in meshes])])
    for p in range(1, 5):
        ks = sorted((k for k in range(len(meshes)) if meshes[k].p == p),
                    key=lambda k: meshes[k].n_elem)[:2]
        for k in ks:
            m = meshes[k]
            v, e = fields[k]
            S = O.qdata(m.elem_nodes, p, qs[k], m.n_nodes, m.x0, m.x0, v, e)["S"]
            yo = O.force_mult(m.elem_nodes, p, qs[k], m.n_nodes, S)
            ya = O.force_mult(m.elem_nodes, p, qs[k], m.n_nodes, S, absmode=True)
            assert rel_cw(y1[:, noff[k]:noff[k + 1]], yo, ya) < TOL, (k, p)


def test_each_mesh_runs_its_own_cg(torch_cuda):
    """Meshes of very different element sizes (and so mass-matrix scales) in one
    context: every mesh converges with its own CG scalars, in about as many
    iterations as it needs alone, and the iteration limit is reported."""
    t = torch_cuda
    # two meshes of one class, each of several patches (the class's workgroups are
    # remapped across XCDs, so a mesh's partials must follow its patches)
    cases = [make_case(3, 2, 4, seed=61), make_case(6, 2, 4, seed=62), make_case(2, 3, 5, seed=63),
             make_case(1, 2, 4, seed=64)]
    rng = np.random.default_rng(9)
    xs = [rng.standard_normal((3, c.N)) for c in cases]
    bs = [O.mass_mult(c.mesh.elem_nodes, c.p, c.Q, c.N, oracle_qdata(c)["mq"], xk)
          for c, xk in zip(cases, xs)]
    alone = []
    for c, b in zip(cases, bs):
        g1 = Multi(t, [c.mesh], [c.Q], 0)
        xg = t.zeros((3, c.N), dtype=t.float64, device="cuda")
        rc, it, rr = fe.fe_mass_cg(g1.ctx, dev(t, b), xg, None, rel_tol=1e-12)
        assert rc == fe.FE_OK
        alone.append(it)
    for flags in (0, B | G):
        g = Multi(t, [c.mesh for c in cases], [c.Q for c in cases], flags)
        xg = t.zeros((3, g.Ntot), dtype=t.float64, device="cuda")
        rc, it, rr = fe.fe_mass_cg(g.ctx, g.h1(bs), xg, None, rel_tol=1e-12)
        assert rc == fe.FE_OK and rr <= 1e-12
        assert abs(it - max(alone)) <= 2, (it, alone)
        xh = xg.cpu().numpy()
        for k, xk in enumerate(xs):
            assert np.linalg.norm(g.h1_slice(xh, k) - xk) < 1e-9 * np.linalg.norm(xk), k
        # stopped by the iteration limit after an odd and an even count: every
        # mesh's x is its own k-th CG iterate (the last direction may have been
        # left pending by the step and is added after the loop)
        for k_it in (3, 2):
            xg.zero_()
            rc, it, rr = fe.fe_mass_cg(g.ctx, g.h1(bs), xg, None, rel_tol=1e-12, max_iter=k_it,
                                       check=False)
            assert rc == fe.FE_ENOTCONV and it == k_it
            xh = xg.cpu().numpy()
            for k, (c, b) in enumerate(zip(cases, bs)):
                xo, ito, _, ok = O.mass_cg(c.mesh.elem_nodes, c.p, c.Q, c.N, oracle_qdata(c)["mq"], b,
                                           rel_tol=1e-12, max_iter=k_it)
                assert not ok and ito == k_it
                assert np.linalg.norm(g.h1_slice(xh, k) - xo) <= 1e-11 * np.linalg.norm(xo), (k, k_it)
