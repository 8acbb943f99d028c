"""Pins of the oracle's multi-material quadrature data (Sec. 2.1's
multi-material equations; Sec. 3.3's -sum_k F_k 1, M_E,k de_k/dt = F_k^T v and
eta_k rho_k |J| = eta_k0 rho_k0 |J0|): S_k = w detJ eta_k sigma_k J^-T.

Each test ties it to something other than itself: the pinned single-material
routine (one material of volume fraction 1, and a mixture of materials in
one state, which the ideal gas makes linear in the densities), the closed-form
free-stream face sums on a dilated mesh, the discrete energy exchange, an
affine volume-fraction field checked point by point on an unperturbed mesh,
and linearity in the volume fractions.
"""
import numpy as np
import pytest

import oracle as O
from paper_2112_07075_amd import workload as W

GAMMA = 5.0 / 3.0


def moved(mesh, scale=0.03, seed=3):
    rng = np.random.default_rng(seed)
    inner = (mesh.ref > 0) * (mesh.ref < 1)
    return mesh.x0 + scale / mesh.n * rng.uniform(-1, 1, mesh.x0.shape) * inner


@pytest.mark.parametrize("p", [1, 2, 3])
def test_one_material_of_fraction_one_is_the_single_material_data(p):
    Q = p + 2
    mesh = W.cube_mesh(2, p, W.default_amp(p), seed=21)
    v, e = W.taylor_green_fields(mesh)
    v = v - 0.3 * (mesh.x0 - 0.5)
    x = moved(mesh)
    M, N = mesh.elem_nodes, mesh.n_nodes
    ref = O.qdata(M, p, Q, N, mesh.x0, x, v, e, rho0=1.3, gamma=1.4)["S"]
    S = O.qdata_mm(M, p, Q, N, mesh.x0, x, v, e[None], np.ones((1,) + e.shape), [1.4], [1.3])
    scale = np.abs(ref).max()
    assert np.abs(S[0] - ref).max() < 1e-14 * scale


def test_mixture_in_one_state_sums_to_the_mixture_density():
    # same gamma and energy, constant fractions a and 1-a: the pressure and
    # the viscosity are linear in the density, so S_1 + S_2 is the single-
    # material S of density a rho_1 + (1-a) rho_2
    p, Q, a = 2, 4, 0.3
    mesh = W.cube_mesh(3, p, 0.1, seed=22)
    v, e = W.taylor_green_fields(mesh)
    v = v - 0.3 * (mesh.x0 - 0.5)
    x = moved(mesh)
    M, N = mesh.elem_nodes, mesh.n_nodes
    eta = np.stack([np.full_like(e, a), np.full_like(e, 1 - a)])
    S = O.qdata_mm(M, p, Q, N, mesh.x0, x, v, np.stack([e, e]), eta, [GAMMA, GAMMA], [2.0, 0.5])
    ref = O.qdata(M, p, Q, N, mesh.x0, x, v, e, rho0=a * 2.0 + (1 - a) * 0.5)["S"]
    assert np.abs(S[0] + S[1] - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_free_stream_faces_per_material_on_a_dilated_mesh(p):
    # v = 0, uniform e_k, constant eta_k, x = s x0: sigma_k = -p_k I with
    # rho_k = rho_k0 / s^3; the faces x_c = s carry -eta_k p_k s^2 in total and
    # interior nodes nothing
    Q, s = p + 2, 1.25
    mesh = W.cube_mesh(2, p, W.default_amp(p), seed=23)
    M, N = mesh.elem_nodes, mesh.n_nodes
    E = mesh.n_elem
    gam, rho0, e0, eta = [1.4, 3.0], [1.0, 7.0], [2.0, 0.5], [0.25, 0.75]
    e = np.stack([np.full((E, p ** 3), v) for v in e0])
    et = np.stack([np.full((E, p ** 3), v) for v in eta])
    S = O.qdata_mm(M, p, Q, N, mesh.x0, s * mesh.x0, np.zeros_like(mesh.x0), e, et, gam, rho0)
    bnd = ((mesh.ref == 0.0) | (mesh.ref == 1.0)).any(axis=0)
    for k in range(2):
        y = O.force_mult(M, p, Q, N, S[k])
        pk = (gam[k] - 1.0) * rho0[k] / s ** 3 * e0[k]
        for c in range(3):
            assert abs(y[c, mesh.ref[c] == 1.0].sum() + eta[k] * pk * s * s) < 1e-12
            assert abs(y[c, mesh.ref[c] == 0.0].sum() - eta[k] * pk * s * s) < 1e-12
        assert np.abs(y[:, ~bnd]).max() < 1e-12


def test_energy_exchange_over_materials():
    p, Q = 2, 4
    mesh = W.cube_mesh(3, p, 0.1, seed=24)
    v, e = W.taylor_green_fields(mesh)
    v = v - 0.2 * (mesh.x0 - 0.5)
    M, N = mesh.elem_nodes, mesh.n_nodes
    rng = np.random.default_rng(4)
    eta1 = rng.uniform(0.1, 0.9, e.shape)
    S = O.qdata_mm(M, p, Q, N, mesh.x0, moved(mesh), v, np.stack([e, 0.5 * e]),
                   np.stack([eta1, 1 - eta1]), [GAMMA, 1.4], [1.0, 3.0])
    mom = sum(float((v * O.force_mult(M, p, Q, N, S[k])).sum()) for k in range(2))
    ene = sum(float(O.force_mult_T(M, p, Q, N, S[k], v).sum()) for k in range(2))
    scale = sum(float((np.abs(v) * O.force_mult(M, p, Q, N, S[k], absmode=True)).sum())
                for k in range(2))
    assert abs(mom - ene) < 1e-14 * scale


def test_affine_fraction_is_read_point_by_point():
    # unperturbed Q2 mesh: the L2 space Q1 holds eta = a + b.X exactly, so at
    # every point S_k(eta) = eta(X_q) S_k(1), X_q the point's position
    p, Q, n = 2, 4, 2
    mesh = W.cube_mesh(n, p, 0.0)
    M, N, E = mesh.elem_nodes, mesh.n_nodes, mesh.n_elem
    v, e = W.taylor_green_fields(mesh)
    tl, _ = O.gauss_legendre(p)               # L2 nodes
    tq, _ = O.gauss_legendre(Q)
    a, b = 0.2, np.array([0.3, -0.1, 0.25])
    ex, ey, ez = (np.arange(E) % n, (np.arange(E) // n) % n, np.arange(E) // (n * n))
    corner = np.stack([ex, ey, ez], axis=1) / n       # element origin, [E][3]
    idx = np.indices((p, p, p))                        # [jz, jy, jx]
    loc = np.stack([tl[idx[2]], tl[idx[1]], tl[idx[0]]], axis=-1).reshape(-1, 3)
    eta = a + (corner[:, None, :] + loc[None] / n) @ b          # [E][p^3]
    S1 = O.qdata_mm(M, p, Q, N, mesh.x0, mesh.x0, v, e[None], np.ones((1, E, p ** 3)), [GAMMA], [1.0])
    Se = O.qdata_mm(M, p, Q, N, mesh.x0, mesh.x0, v, e[None], eta[None], [GAMMA], [1.0])
    iq = np.indices((Q, Q, Q))
    locq = np.stack([tq[iq[2]], tq[iq[1]], tq[iq[0]]], axis=-1).reshape(-1, 3)
    etaq = a + (corner[:, None, :] + locq[None] / n) @ b          # [E][Q^3]
    ref = S1[0] * etaq[:, None, None, :]
    assert np.abs(Se[0] - ref).max() < 1e-13 * np.abs(ref).max()


def test_linear_in_the_fractions_and_material_masses():
    p, Q = 3, 5
    mesh = W.cube_mesh(2, p, W.default_amp(p), seed=25)
    v, e = W.taylor_green_fields(mesh)
    M, N = mesh.elem_nodes, mesh.n_nodes
    rng = np.random.default_rng(5)
    ea, eb = rng.uniform(0, 0.5, e.shape), rng.uniform(0, 0.5, e.shape)
    x = moved(mesh)
    args = (M, p, Q, N, mesh.x0, x, v, e[None])
    Sa = O.qdata_mm(*args, ea[None], [GAMMA], [2.0])
    Sb = O.qdata_mm(*args, eb[None], [GAMMA], [2.0])
    Sab, mq = O.qdata_mm(*args, (ea + eb)[None], [GAMMA], [2.0], want_mq=True)
    assert np.abs(Sab - Sa - Sb).max() < 1e-13 * np.abs(Sab).max()
    # a constant fraction f: the material's mass is f rho_k0 times the volume (1)
    _, mqc = O.qdata_mm(*args, np.full((1,) + e.shape, 0.4), [GAMMA], [2.0], want_mq=True)
    assert abs(mqc.sum() - 0.4 * 2.0) < 1e-13
