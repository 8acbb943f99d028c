"""Oracle pins for an initial density given at every quadrature point
(Sec. 3.3's pointwise rho |J| = rho0 |J0| with rho0 varying over the mesh).

* m_q = rho0(x0_q) detJ0 w_q, point by point, on an affine (unperturbed) cube
  mesh: the expected value is formed here from the element's corner nodes and
  numpy's Gauss-Legendre rule, with a density that differs along every axis,
  so that an element, point or axis mix-up in the oracle's indexing fails.
* On a uniformly dilated mesh x = s x0 with v = 0 and a constant e, the moment
  sum_i x_i,d (F 1)_i,c equals -delta_cd (gamma - 1) e int rho0 dx0 (the
  ideal-gas pressure integrated over the moved mesh, whose mass is that of
  x0), which pins that S takes rho = rho0(q) detJ0 / detJ point by point.
* A constant rho0_q gives exactly the scalar-rho0 data."""
import numpy as np
import pytest

import oracle as O
from paper_2112_07075_amd import workload as W


def rho0_fn(x, y, z):
    return (1.0 + x) * (2.0 + y * y) * (1.0 + 3.0 * z)


RHO0_INT = 1.5 * (2.0 + 1.0 / 3.0) * 2.5   # its integral over [0,1]^3


def points_and_jac(mesh, p, Q):
    """Physical Gauss points [E][3][Q^3] (q = qx + Q (qy + Q qz)) and detJ0 [E]
    of the affine elements, from the corner nodes."""
    D = p + 1
    t, wt = np.polynomial.legendre.leggauss(Q)
    xi, w1 = 0.5 * (t + 1.0), 0.5 * wt
    M = mesh.elem_nodes
    x0 = mesh.x0
    c0 = x0[:, M[:, 0]]                              # [3][E]
    ex = x0[:, M[:, D - 1]] - c0
    ey = x0[:, M[:, D * (D - 1)]] - c0
    ez = x0[:, M[:, D * D * (D - 1)]] - c0
    qz, qy, qx = np.meshgrid(np.arange(Q), np.arange(Q), np.arange(Q), indexing="ij")
    qx, qy, qz = qx.ravel(), qy.ravel(), qz.ravel()
    pts = (c0[:, :, None] + ex[:, :, None] * xi[qx] + ey[:, :, None] * xi[qy] +
           ez[:, :, None] * xi[qz]).transpose(1, 0, 2)
    J = np.stack([ex, ey, ez], axis=-1).transpose(1, 0, 2)   # [E][3][3]
    w = w1[qx] * w1[qy] * w1[qz]
    return pts, np.linalg.det(J), w


@pytest.mark.parametrize("p,Q", [(1, 2), (2, 4), (3, 5)])
def test_point_mass_is_rho0_detJ0_w(p, Q):
    mesh = W.cube_mesh(3, p, 0.0, seed=5, permute_seed=p)
    pts, dJ, w = points_and_jac(mesh, p, Q)
    r0 = rho0_fn(pts[:, 0], pts[:, 1], pts[:, 2])          # [E][Q^3]
    E = mesh.elem_nodes.shape[0]
    x0 = mesh.x0
    e = np.full((E, p ** 3), 2.0)
    qd = O.qdata(mesh.elem_nodes, p, Q, x0.shape[1], x0, x0, None, e, rho0=r0, want=("mq",))
    ref = r0 * dJ[:, None] * w[None, :]
    # rounding: two computations of the Gauss rule and of detJ0 (sum over nodes)
    assert np.abs(qd["mq"] - ref).max() < 1e-13 * np.abs(ref).max()
    # the masses add up to int rho0 over the cube (Q >= 2 integrates rho0 exactly)
    assert abs(qd["mq"].sum() - RHO0_INT) < 1e-13 * RHO0_INT


@pytest.mark.parametrize("p,Q", [(1, 3), (2, 4), (3, 5)])
def test_dilated_free_stream_pressure_moment(p, Q):
    mesh = W.cube_mesh(2, p, 0.0, seed=6)
    pts, _, _ = points_and_jac(mesh, p, Q)
    r0 = rho0_fn(pts[:, 0], pts[:, 1], pts[:, 2])
    E, N = mesh.elem_nodes.shape[0], mesh.x0.shape[1]
    s, e0, gam = 1.3, 0.7, 1.4
    x = s * mesh.x0
    e = np.full((E, p ** 3), e0)
    qd = O.qdata(mesh.elem_nodes, p, Q, N, mesh.x0, x, np.zeros_like(x), e, rho0=r0, gamma=gam,
                 want=("S",))
    y = O.force_mult(mesh.elem_nodes, p, Q, N, qd["S"])     # [3][N]
    mom = x @ y.T                                          # [d][c] = sum_i x_i,d y_i,c
    ref = -(gam - 1.0) * e0 * RHO0_INT * np.eye(3)
    assert np.abs(mom - ref).max() < 1e-12 * abs(ref[0, 0])


def test_constant_rho0_q_is_scalar_rho0():
    c_mesh = W.cube_mesh(2, 2, 0.08, seed=7)
    E, N = c_mesh.elem_nodes.shape[0], c_mesh.x0.shape[1]
    v, e = W.taylor_green_fields(c_mesh)
    x = c_mesh.x0 + 0.02 * v
    a = O.qdata(c_mesh.elem_nodes, 2, 4, N, c_mesh.x0, x, v, e, rho0=2.5, want=("S", "mq", "dt"))
    b = O.qdata(c_mesh.elem_nodes, 2, 4, N, c_mesh.x0, x, v, e, rho0=np.full((E, 64), 2.5),
                want=("S", "mq", "dt"))
    for k in ("S", "mq", "dt"):
        assert np.array_equal(a[k], b[k])
