"""Pins of the oracle's stiffness (diffusion) operator, the extra operator the
hyper-viscosity term needs (Sec. 2.1; the diffusion integrator of Sec. 6):
K[i][j] = int kappa grad w_i . grad w_j dx on the current mesh, per component.

Each test ties the oracle to something other than itself: the closed-form 1-D
stiffness and mass matrices of quadratic Lagrange functions, the divergence
theorem for linear fields (exact quadrature), the constant null space,
invariance under rigid motion and the scaling of the operator under
dilation, and a 1-D tensor factorisation for a point-dependent coefficient.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O
from paper_2112_07075_amd import workload as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))

# 1-D stiffness of the quadratic Lagrange functions at {0, 1/2, 1} on [0, 1]:
# derivatives 4t-3, 4-8t, 4t-1; int (4t-3)^2 = 7/3, int (4t-3)(4-8t) = -8/3,
# int (4t-3)(4t-1) = 1/3, int (4-8t)^2 = 16/3.
K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]], dtype=np.float64) / 3.0


def m1():
    return np.array([[float(Fr(s)) for s in row] for row in GOLD["mass_1d_q2_gll"]["M1"]])


def kron3(az, ay, ax):
    # local index i = ix + D (iy + D iz): x fastest
    return np.kron(az, np.kron(ay, ax))


@pytest.mark.parametrize("Q", [3, 4, 5])
def test_unperturbed_q2_element_is_the_tensor_closed_form(Q):
    n = 2
    mesh = W.cube_mesh(n, 2, 0.0)
    h = 1.0 / n
    M1 = m1()
    ref = h * (kron3(M1, M1, K1) + kron3(M1, K1, M1) + kron3(K1, M1, M1))
    for el in (0, 5):
        KE = O.stiff_elem_matrix(2, Q, mesh.elem_nodes[el], mesh.x0)
        np.testing.assert_allclose(KE, ref, rtol=0, atol=2e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_constants_are_the_null_space_on_moved_meshes(p):
    mesh = W.cube_mesh(3, p, W.default_amp(p), seed=11)
    rng = np.random.default_rng(5)
    x = mesh.x0 + 0.02 / 3 * rng.uniform(-1, 1, mesh.x0.shape) * (mesh.ref > 0) * (mesh.ref < 1)
    N, M, Q = mesh.n_nodes, mesh.elem_nodes, p + 2
    ones = np.ones((3, N))
    y = O.stiff_mult(M, p, Q, N, x, ones)
    scale = O.stiff_mult(M, p, Q, N, x, ones, absmode=True).max()
    assert np.abs(y).max() < 1e-14 * scale
    KE = O.stiff_elem_matrix(p, Q, M[7], x)
    np.testing.assert_allclose(KE, KE.T, rtol=0, atol=1e-15 * np.abs(KE).max())
    assert np.linalg.eigvalsh(KE).min() > -1e-13 * np.abs(KE).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_linear_field_divergence_theorem(p):
    # u = x_c (exact in the isoparametric H1 space): (K u)_g = boundary integral
    # of w_g n_c, so interior rows vanish, and the rows of the nodes on the face
    # x_c = 1 sum to its area (1), those on x_c = 0 to -1. detJ-weighted
    # integrands have degree 3p-1 per variable, exact with Q = p+2 points.
    mesh = W.cube_mesh(3, p, W.default_amp(p), seed=12)
    N, M, Q = mesh.n_nodes, mesh.elem_nodes, p + 2
    x = mesh.x0
    y = O.stiff_mult(M, p, Q, N, x, x)            # all three components: u_c = x_c
    scale = O.stiff_mult(M, p, Q, N, x, x, absmode=True).max()
    bnd = ((mesh.ref == 0.0) | (mesh.ref == 1.0)).any(axis=0)
    assert np.abs(y[:, ~bnd]).max() < 1e-13 * scale
    for c in range(3):
        top = mesh.ref[c] == 1.0
        bot = mesh.ref[c] == 0.0
        assert abs(y[c, top].sum() - 1.0) < 1e-13
        assert abs(y[c, bot].sum() + 1.0) < 1e-13
        # the energy of a unit gradient over the unit volume
        assert abs(float(x[c] @ y[c]) - 1.0) < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_rigid_motion_invariance_and_dilation_scaling(p):
    mesh = W.cube_mesh(2, p, W.default_amp(p), seed=13)
    N, M, Q = mesh.n_nodes, mesh.elem_nodes, p + 2
    rng = np.random.default_rng(6)
    u = rng.standard_normal((3, N))
    y0 = O.stiff_mult(M, p, Q, N, mesh.x0, u)
    scale = O.stiff_mult(M, p, Q, N, mesh.x0, u, absmode=True).max()
    # rotation about a skew axis plus a shift: K is unchanged
    a = np.array([1.0, 2.0, -0.5])
    a /= np.linalg.norm(a)
    th = 0.7
    Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    xr = R @ mesh.x0 + np.array([[0.3], [-1.0], [2.0]])
    assert np.abs(O.stiff_mult(M, p, Q, N, xr, u) - y0).max() < 1e-13 * scale
    # dilation by s: gradients scale by 1/s, volume by s^3, so K scales by s
    s = 1.7
    assert np.abs(O.stiff_mult(M, p, Q, N, s * mesh.x0, u) - s * y0).max() < 1e-13 * scale
    # a shear is not a rigid motion: K changes
    A = np.array([[1.0, 0.4, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    assert np.abs(O.stiff_mult(M, p, Q, N, A @ mesh.x0, u) - y0).max() > 1e-3 * scale


@pytest.mark.parametrize("axis", [0, 2])
def test_point_coefficient_factorises_on_an_unperturbed_element(axis):
    # kappa_q = f(t) of one coordinate only, on the unit cube element (p = 2):
    # K_E = sum over the derivative direction of 1-D matrices, the axis of f
    # taking the f-weighted 1-D stiffness / mass. Checks that kappa is read
    # per point in the lexicographic order q = qx + Q (qy + Q qz).
    p, Q = 2, 4
    mesh = W.cube_mesh(1, p, 0.0)
    t, w = O.gauss_legendre(Q)
    f = 1.0 + t ** 2 + 0.5 * t
    nodes = O.gll_nodes(p)
    B = np.array([O.lagrange(nodes, tq)[0] for tq in t])    # [q][a]
    G = np.array([O.lagrange(nodes, tq)[1] for tq in t])
    Mw = lambda c: (B * (w * c)[:, None]).T @ B
    Kw = lambda c: (G * (w * c)[:, None]).T @ G
    one = np.ones(Q)
    fx = [f if axis == d else one for d in range(3)]       # coefficient factor per axis
    ref = (kron3(Mw(fx[2]), Mw(fx[1]), Kw(fx[0])) + kron3(Mw(fx[2]), Kw(fx[1]), Mw(fx[0])) +
           kron3(Kw(fx[2]), Mw(fx[1]), Mw(fx[0])))
    idx = np.indices((Q, Q, Q))                               # [qz, qy, qx]
    tq = [t[idx[2]], t[idx[1]], t[idx[0]]]                    # coordinate of each point per axis
    kap = (1.0 + tq[axis] ** 2 + 0.5 * tq[axis]).ravel()     # q = qx + Q (qy + Q qz)
    KE = O.stiff_elem_matrix(p, Q, mesh.elem_nodes[0], mesh.x0, kap)
    np.testing.assert_allclose(KE, ref, rtol=0, atol=1e-14)
    # and an elementwise constant coefficient scales the element's contribution
    KE2 = O.stiff_elem_matrix(p, Q, mesh.elem_nodes[0], mesh.x0, np.full(Q ** 3, 2.5))
    np.testing.assert_allclose(KE2, 2.5 * O.stiff_elem_matrix(p, Q, mesh.elem_nodes[0], mesh.x0),
                               rtol=0, atol=1e-14)
