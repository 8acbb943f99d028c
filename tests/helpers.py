"""Shared helpers of the tests: synthetic cases, oracle references and error measures."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle as O
from paper_2112_07075_amd import workload as W


@dataclass
class Case:
    n: int
    p: int
    Q: int
    mesh: W.Mesh
    x: np.ndarray   # current positions [3][N]
    v: np.ndarray   # [3][N]
    e: np.ndarray   # [E][p^3]
    q1: float
    q2: float

    @property
    def N(self):
        return self.mesh.n_nodes

    @property
    def E(self):
        return self.mesh.n_elem


def make_case(n, p, Q=None, amp=None, seed=0, permute=None, q1=0.5, q2=2.0, move=0.05,
              compress=0.0) -> Case:
    """Perturbed cube with Taylor-Green fields. The current positions are x0 moved by
    move*h*v, so rho = rho0 detJ0/detJ differs from rho0. compress adds -compress*(x-1/2)
    to v, which switches on the quadratic viscosity term."""
    Q = Q or p + 2
    amp = W.default_amp(p) if amp is None else amp
    mesh = W.cube_mesh(n, p, amp, seed=seed, permute_seed=permute)
    v, e = W.taylor_green_fields(mesh)
    if compress:
        v = v - compress * (mesh.x0 - 0.5)
    x = mesh.x0 + move * (1.0 / n) * v
    return Case(n, p, Q, mesh, np.ascontiguousarray(x), np.ascontiguousarray(v), e, q1, q2)


def oracle_qdata(c: Case, elems=None):
    return O.qdata(c.mesh.elem_nodes, c.p, c.Q, c.N, c.mesh.x0, c.x, c.v, c.e, q1=c.q1, q2=c.q2,
                   elems=elems)


def elems_touching(mesh: W.Mesh, nodes) -> np.ndarray:
    return np.nonzero(np.isin(mesh.elem_nodes, nodes).any(axis=1))[0].astype(np.int32)


def rel_cw(got, ref, absref) -> float:
    """max |got - ref| / max (|F||e|): errors on the scale of the sum of term magnitudes."""
    got, ref, absref = (np.asarray(a, dtype=np.float64).ravel() for a in (got, ref, absref))
    den = np.abs(absref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def rel_2(got, ref) -> float:
    got, ref = np.asarray(got).ravel(), np.asarray(ref).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def rel_elem(got, ref) -> float:
    """Entrywise error normalised by each element's largest reference magnitude."""
    got = np.asarray(got).reshape(ref.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    scale[scale == 0] = 1.0
    return float((np.abs(got - ref) / scale).max())
