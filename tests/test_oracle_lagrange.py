"""Pins of the oracle's full Lagrange step (the semi-discrete system of
Sec. 3.3 advanced by a two-stage scheme), against what the mathematics fixes:
closed forms of the thermodynamic mass matrix and of the stable time step,
the steady still gas, exact total-energy and momentum conservation, and the
second-order convergence of the two-stage scheme."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2112_07075_amd import workload as W

GAMMA = 5.0 / 3.0


def gl_weights3(n):
    _, w = np.polynomial.legendre.leggauss(n)
    w = 0.5 * w
    return np.einsum("i,j,k->kji", w, w, w).ravel()


def tg_state(n, p, amp, seed):
    m = W.cube_mesh(n, p, amp, seed=seed)
    v, e = W.taylor_green_fields(m)
    ess = W.boundary_normal_dofs(m)
    v.ravel()[ess] = 0.0            # v.n = 0 holds exactly on the walls
    return m, v, e, ess


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5), (4, 6)])
def test_l2_mass_closed_form(p, Q):
    # axis-aligned elements of side h: M_E = rho0 h^3 (M1 x M1 x M1) with the 1-D
    # mass of the Lagrange basis at the p Gauss points, which is diagonal with the
    # p-point Gauss weights (the p-point rule integrates phi_j phi_k exactly)
    n, rho0 = 2, 1.7
    h = 1.0 / n
    m = W.cube_mesh(n, p, amp=0.0)
    mq = O.qdata(m.elem_nodes, p, Q, m.n_nodes, m.x0, m.x0, None, None, rho0=rho0,
                 want=("mq",))["mq"]
    ME = O.l2_mass(m.elem_nodes, p, Q, mq)
    expect = rho0 * h ** 3 * np.diag(gl_weights3(p))
    for el in range(m.n_elem):
        np.testing.assert_allclose(ME[el], expect, rtol=0, atol=4e-15 * expect.max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_l2_mass_perturbed_spd_and_total(p):
    # the basis is a partition of unity, so 1^T M_E 1 is the element's mass and the
    # masses add up to rho0 |Omega| = 1; every M_E is symmetric positive definite
    Q = p + 2
    m = W.cube_mesh(2, p, W.default_amp(p), seed=21)
    mq = O.qdata(m.elem_nodes, p, Q, m.n_nodes, m.x0, m.x0, None, None, want=("mq",))["mq"]
    ME = O.l2_mass(m.elem_nodes, p, Q, mq)
    np.testing.assert_allclose(ME.sum(axis=(1, 2)), mq.sum(axis=1), rtol=1e-14)
    assert abs(ME.sum() - 1.0) < 1e-14
    assert np.abs(ME - ME.transpose(0, 2, 1)).max() < 1e-18
    assert np.linalg.eigvalsh(ME).min() > 0


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("s", [1.0, 1.2])
def test_time_step_closed_form(p, s):
    # x = s x0 on an axis-aligned mesh, v = -k (x - c), e = e0: rho = 1/s^3,
    # l = s h / p, c_s = sqrt(gamma (gamma-1) e0) and tr eps = -3k everywhere, so
    # every point's step is l / ((1+q1) c_s + 3 q2 l k)
    Q, n, k, e0, q1, q2 = p + 2, 2, 0.7, 3.0, 0.5, 2.0
    h = 1.0 / n
    m = W.cube_mesh(n, p, amp=0.0)
    x = s * m.x0
    v = -k * (x - 0.5)
    e = np.full((m.n_elem, p ** 3), e0)
    dt = O.qdata(m.elem_nodes, p, Q, m.n_nodes, m.x0, x, v, e, q1=q1, q2=q2, want=("dt",))["dt"]
    ell = s * h / p
    cs = math.sqrt(GAMMA * (GAMMA - 1.0) * e0)
    np.testing.assert_allclose(dt, ell / ((1 + q1) * cs + 3 * q2 * ell * k), rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_still_gas_stays_still(p):
    # v = 0, e = e0 with v.n = 0 walls: the only forces are normal wall forces, which
    # the walls take up, so one step changes nothing (and dt = cfl l_min / ((1+q1) c_s))
    Q = p + 2
    m = W.cube_mesh(3, p, W.default_amp(p), seed=22)
    N = m.n_nodes
    e0 = 3.0
    e = np.full((m.n_elem, p ** 3), e0)
    ess = W.boundary_normal_dofs(m)
    x1, v1, e1, dt = O.lagrange_step(m.elem_nodes, p, Q, N, m.x0, m.x0, np.zeros((3, N)), e,
                                     ess=ess, cfl=0.5)
    detJ = O.qdata(m.elem_nodes, p, Q, N, m.x0, m.x0, None, None, want=("detJ",))["detJ"]
    cs = math.sqrt(GAMMA * (GAMMA - 1.0) * e0)
    assert abs(dt - 0.5 * (np.cbrt(detJ.min()) / p) / (1.5 * cs)) < 1e-15
    assert np.abs(v1).max() < 1e-12 * (GAMMA - 1.0) * e0 * dt * 3   # scale p0 dt / h
    assert np.abs(e1 - e0).max() < 1e-13 * e0
    assert np.abs(x1 - m.x0).max() < 1e-16


@pytest.mark.parametrize("p", [1, 2, 3])
def test_step_conserves_total_energy(p):
    # kinetic energy lost by the midpoint forces equals internal energy gained:
    # vbar^T M_v (v' - v) = -dt vbar^T F 1 and 1^T M_E (e' - e) = dt 1^T F^T vbar
    Q = p + 2
    m, v, e, ess = tg_state(3, p, W.default_amp(p), seed=23)
    N = m.n_nodes
    M = m.elem_nodes
    mq = O.qdata(M, p, Q, N, m.x0, m.x0, None, None, want=("mq",))["mq"]
    k0, i0 = O.total_energy(M, p, Q, N, mq, v, e)
    x1, v1, e1, dt = O.lagrange_step(M, p, Q, N, m.x0, m.x0, v, e, ess=ess, cfl=0.5)
    k1, i1 = O.total_energy(M, p, Q, N, mq, v1, e1)
    assert abs(k1 - k0) > 1e-6 * k0       # energy really moved between the two kinds
    assert abs((k1 + i1) - (k0 + i0)) < 1e-13 * (k0 + i0)
    assert np.all(v1.ravel()[ess] == 0.0)


def test_step_conserves_momentum_without_walls():
    # with no essential DOFs, 1^T M_v (v' - v) = -dt 1^T F 1 = 0 for each component
    p, Q = 2, 4
    m = W.cube_mesh(2, p, 0.1, seed=24)
    N = m.n_nodes
    M = m.elem_nodes
    v, e = W.taylor_green_fields(m)
    v = v + np.array([[0.3], [-0.1], [0.2]])
    mq = O.qdata(M, p, Q, N, m.x0, m.x0, None, None, want=("mq",))["mq"]
    P0 = O.mass_mult(M, p, Q, N, mq, v).sum(axis=1)
    _, v1, _, dt = O.lagrange_step(M, p, Q, N, m.x0, m.x0, v, e, cfl=0.5)
    P1 = O.mass_mult(M, p, Q, N, mq, v1).sum(axis=1)
    assert np.abs(P1 - P0).max() < 1e-13 * np.abs(P0).max()
    assert np.abs(v1 - v).max() > 1e-3 * dt   # the walls are free to move: forces act


def test_two_stage_scheme_is_second_order():
    # the state at T = 2 dt0 from steps of dt0 and dt0/2 against 32 steps of dt0/16:
    # halving the step divides the error by about 4
    p, Q = 2, 4
    m, v, e, ess = tg_state(2, p, 0.1, seed=25)
    N, M = m.n_nodes, m.elem_nodes
    dt0 = 0.01

    def run(nsteps, dt):
        x, vv, ee = m.x0.copy(), v.copy(), e.copy()
        for _ in range(nsteps):
            x, vv, ee, used = O.lagrange_step(M, p, Q, N, m.x0, x, vv, ee, ess=ess, cfl=10.0,
                                              dt_max=dt)
            assert used == dt
        return np.concatenate([x.ravel(), vv.ravel(), ee.ravel()])

    ref = run(32, dt0 / 16)
    e1 = np.abs(run(2, dt0) - ref).max()
    e2 = np.abs(run(4, dt0 / 2) - ref).max()
    rate = math.log2(e1 / e2)
    assert 1.8 < rate < 2.4, (e1, e2, rate)
