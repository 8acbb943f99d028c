"""Seeded synthetic inputs: perturbed unit-cube hex meshes and Taylor-Green fields.

This module produces *input arrays only*. It contains none of the operator
arithmetic (no basis tables, quadrature, Jacobians or contractions); the GPU
library and the CPU oracle each implement that on their own and both consume
the arrays made here.

Layouts (shared by every consumer):
  * scalar H1 nodes of one mesh: lexicographic on the (p*n+1)^3 grid, x fastest
    (optionally renumbered by a seeded random permutation);
  * element e = ex + n*(ey + n*ez); local H1 node i = ix + D*(iy + D*iz), D = p+1;
  * vectors are SoA by component: x[c*N + g];
  * L2 (discontinuous, order p-1) values: e[E][Dl^3], Dl = p, local
    j = jx + Dl*(jy + Dl*jz).

Node placement follows the paper's setting of curved high-order hexahedra
(Sec. 3.2 tensor-product bases; Sec. 2.1 continuous kinematic space): the H1
nodes of each element sit at the Gauss-Lobatto points of [0,1] mapped to the
element, and every node (vertex or high-order) is moved by seeded uniform noise
of +-amp*h in each Cartesian component unless the node lies on that
component's boundary plane, so the domain stays the unit cube.

Random draws use a counter-based splitmix64: draw k of seed s is
mix64(s + (k+1)*0x9E3779B97F4A7C15), converted to a 53-bit uniform in [0,1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Counter-based splitmix64 (Steele, Lea, Flood 2014) of draw indices."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counters.astype(np.uint64) + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """53-bit uniforms in [0, 1) from splitmix64 draws."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def lobatto_points01(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto points on [0,1]: the ends plus the roots of P_p'."""
    if p < 1:
        raise ValueError("order must be >= 1")
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.zeros(0)
    s = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (s + 1.0)


def gauss_points01(n: int) -> np.ndarray:
    """n Gauss-Legendre points on [0,1] (numpy's leggauss, mapped)."""
    s, _ = np.polynomial.legendre.leggauss(n)
    return 0.5 * (s + 1.0)


@dataclass
class Mesh:
    n: int                 # elements per edge
    p: int                 # H1 order
    amp: float             # perturbation amplitude, in units of h
    seed: int
    n_elem: int
    n_nodes: int
    elem_nodes: np.ndarray  # int32 [E][D^3]
    x0: np.ndarray          # float64 [3][N]
    ref: np.ndarray         # float64 [3][N] unperturbed positions
    perm: np.ndarray | None = None  # old id -> new id, if renumbered
    extra: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return self.p + 1


def cube_mesh(n: int, p: int, amp: float = 0.1, seed: int = 0,
              permute_seed: int | None = None, vertex_amp: float | None = None) -> Mesh:
    """Structured n^3 hex mesh of [0,1]^3 with order-p nodes, seeded perturbation.

    Every node component moves by amp*h*(2u-1) (u uniform in [0,1) from
    splitmix64 of (seed, 3g+c)) unless the node lies on that component's
    boundary plane. With vertex_amp, the element vertices instead move by
    vertex_amp*h*(2u-1), every other node follows the trilinear map of its
    element's moved vertices and then moves by amp*h*(2u-1) of its own (so the
    elements stay curved): vertex noise of a larger amplitude than independent
    high-order node noise allows without inverting elements."""
    if n < 1 or p < 1:
        raise ValueError("n and p must be >= 1")
    D = p + 1
    M = p * n + 1
    t = lobatto_points01(p)
    coords = np.empty(M)
    for k in range(n):
        coords[p * k:p * k + D] = (k + t) / n
    coords[0], coords[-1] = 0.0, 1.0
    gz, gy, gx = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
    gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
    N = M ** 3
    ref = np.stack([coords[gx], coords[gy], coords[gz]])
    x0 = ref.copy()
    h = 1.0 / n
    if amp != 0.0 or vertex_amp:
        gidx = np.arange(N, dtype=np.int64)
        if vertex_amp:
            # vertex displacements on the (n+1)^3 vertex grid, then their
            # trilinear interpolation at every node of the element holding it
            vert = (gx % p == 0) & (gy % p == 0) & (gz % p == 0)
            V = n + 1
            dv = np.zeros((3, V, V, V))
            vg = gidx[vert]
            vx, vy, vz = gx[vert] // p, gy[vert] // p, gz[vert] // p
            for c, gc in enumerate((gx, gy, gz)):
                u = uniform01(seed, 3 * vg + c)
                inner = (gc[vert] > 0) & (gc[vert] < M - 1)
                dv[c, vz, vy, vx] = np.where(inner, vertex_amp * h * (2.0 * u - 1.0), 0.0)
            ex_, ey_, ez_ = (np.minimum(gq // p, n - 1) for gq in (gx, gy, gz))
            tx, ty, tz = (t[gq - p * eq] for gq, eq in ((gx, ex_), (gy, ey_), (gz, ez_)))
            disp = np.zeros((3, N))
            for a in (0, 1):
                for b in (0, 1):
                    for d in (0, 1):
                        wgt = ((tx if a else 1 - tx) * (ty if b else 1 - ty) * (tz if d else 1 - tz))
                        disp += wgt * dv[:, ez_ + d, ey_ + b, ex_ + a]
        for c, gc in enumerate((gx, gy, gz)):
            u = uniform01(seed, 3 * gidx + c)
            inner = (gc > 0) & (gc < M - 1)
            own = amp * h * (2.0 * u - 1.0)
            if vertex_amp:
                own = np.where(vert, 0.0, own) + disp[c]
            x0[c] = np.where(inner, ref[c] + own, ref[c])
    # element -> node map, local lexicographic (x fastest)
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    iz, iy, ix = np.meshgrid(np.arange(D), np.arange(D), np.arange(D), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    gmap = ((p * ex[:, None] + ix[None, :])
            + M * ((p * ey[:, None] + iy[None, :]) + M * (p * ez[:, None] + iz[None, :])))
    perm = None
    if permute_seed is not None:
        keys = splitmix64(permute_seed, np.arange(N, dtype=np.int64))
        order = np.argsort(keys, kind="stable")      # new id -> old id
        perm = np.empty(N, dtype=np.int64)
        perm[order] = np.arange(N)                   # old id -> new id
        gmap = perm[gmap]
        x0 = x0[:, order]
        ref = ref[:, order]
    return Mesh(n=n, p=p, amp=amp, seed=seed, n_elem=n ** 3, n_nodes=N,
                elem_nodes=np.ascontiguousarray(gmap, dtype=np.int32),
                x0=np.ascontiguousarray(x0), ref=np.ascontiguousarray(ref), perm=perm)


# ---------------------------------------------------------------- Taylor-Green
GAMMA = 5.0 / 3.0


def tg_velocity(x: np.ndarray) -> np.ndarray:
    """3-D Taylor-Green vortex velocity on [0,1]^3 at points x[3][...]."""
    X, Y, Z = np.pi * x[0], np.pi * x[1], np.pi * x[2]
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z),
                     -np.cos(X) * np.sin(Y) * np.cos(Z),
                     np.zeros_like(X)])


def tg_pressure(x: np.ndarray) -> np.ndarray:
    """Taylor-Green pressure with a background of 100 (low Mach)."""
    X, Y, Z = 2 * np.pi * x[0], 2 * np.pi * x[1], 2 * np.pi * x[2]
    return 100.0 + ((np.cos(X) + np.cos(Y)) * (np.cos(Z) + 2.0) - 2.0) / 16.0


def tg_energy(x: np.ndarray, gamma: float = GAMMA, rho: float = 1.0) -> np.ndarray:
    """Specific internal energy of an ideal gas at the Taylor-Green pressure."""
    return tg_pressure(x) / ((gamma - 1.0) * rho)


def l2_node_ref_positions(mesh: Mesh) -> np.ndarray:
    """Unperturbed positions [3][E][Dl^3] of the order-(p-1) L2 nodes (GL points of a p-point rule)."""
    n, p = mesh.n, mesh.p
    tau = gauss_points01(p)
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    jz, jy, jx = np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij")
    ex, ey, ez = ex.ravel()[:, None], ey.ravel()[:, None], ez.ravel()[:, None]
    jx, jy, jz = jx.ravel()[None, :], jy.ravel()[None, :], jz.ravel()[None, :]
    return np.stack([(ex + tau[jx]) / n, (ey + tau[jy]) / n, (ez + tau[jz]) / n])


def taylor_green_fields(mesh: Mesh, gamma: float = GAMMA):
    """Velocity at the (perturbed) H1 nodes and energy at the L2 nodes.

    v is the closed form at each H1 node position. e is the closed form at the
    unperturbed position of each L2 node (the perturbation is at most 0.1h, so
    the field keeps the Taylor-Green shape and value range, e ~ 150 +- 0.4).
    """
    v = np.ascontiguousarray(tg_velocity(mesh.x0))
    e = np.ascontiguousarray(tg_energy(l2_node_ref_positions(mesh), gamma))
    return v, e


def boundary_normal_dofs(mesh: Mesh) -> np.ndarray:
    """DOF indices c*N+g of the v.n = 0 condition: component c of nodes on x_c in {0,1}."""
    N = mesh.n_nodes
    out = []
    for c in range(3):
        g = np.nonzero((mesh.ref[c] == 0.0) | (mesh.ref[c] == 1.0))[0]
        out.append(c * N + g)
    return np.ascontiguousarray(np.sort(np.concatenate(out)), dtype=np.int32)


# ---------------------------------------------------------------- workloads
def default_amp(p: int) -> float:
    """Perturbation amplitude in units of h: 0.1 for p <= 2, 0.05 for p = 3, 0.025 for p = 4.

    Every node (vertex or high-order) moves independently, so the amplitude has to
    shrink with the Gauss-Lobatto node gap (0.5h at p=2, 0.28h at p=3, 0.17h at
    p=4): +-0.1h at p=3 and +-0.05h at p=4 already invert elements.
    """
    return {1: 0.1, 2: 0.1, 3: 0.05}.get(p, 0.025)


@dataclass
class BatchItem:
    mesh: Mesh
    q1d: int


def batch_meshes(count: int = 256, n_min: int = 4, n_max: int = 24, p_max: int = 4,
                 base_seed: int = 1000) -> list[BatchItem]:
    """Uneven batch of perturbed cubes: per mesh k, seed 1000+k draws n and p; Q = p+2."""
    items = []
    for k in range(count):
        s = base_seed + k
        u = uniform01(s, np.array([1 << 40, (1 << 40) + 1], dtype=np.int64))
        n = n_min + int(math.floor(u[0] * (n_max - n_min + 1)))
        p = 1 + int(math.floor(u[1] * p_max))
        items.append(BatchItem(cube_mesh(n, p, default_amp(p), seed=s), p + 2))
    return items
