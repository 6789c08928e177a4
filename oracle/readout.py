"""Energy and point-probe readouts (oracle, FP64).

Energy: the discrete electromagnetic energy 1/2 sum_k J_k (E^T M E + H^T M H)
summed over the three components (M_k = J_k M, Sec. II-A after eq. (17)).

Probes: a point is assigned to the element that contains it most deeply
(largest smallest barycentric coordinate; lowest element index on exact ties)
and the fields are evaluated with the Lagrange functions at its reference
coordinates.

Parity: pinned by tests/test_oracle_readout.py (energy of a constant field
equals the box volume times the field energy density; probes reproduce
polynomials of degree N exactly).
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh
from .refel import RefElement


def energy(mesh: Mesh, ref: RefElement, q: np.ndarray) -> float:
    EH = q[:, 0:6]
    quad = np.einsum("kci,ij,kcj->k", EH, ref.M, EH)
    return 0.5 * float(np.sum(mesh.J * quad))


def locate(mesh: Mesh, pts: np.ndarray):
    """Element index and reference coordinates of each point."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    elem = np.zeros(len(pts), dtype=np.int64)
    rst = np.zeros((len(pts), 3))
    for i, x in enumerate(pts):
        # r + 1 = Jm^{-1} (x - v0)
        rp1 = np.einsum("kij,kj->ki", mesh.Jinv, x[None, :] - mesh.v[:, 0])
        lam = np.concatenate([1.0 - 0.5 * rp1.sum(axis=1, keepdims=True), 0.5 * rp1], axis=1)
        score = lam.min(axis=1)
        k = int(np.argmax(score))
        if score[k] < -1e-10:
            raise ValueError(f"probe {x} outside the mesh")
        elem[i] = k
        rst[i] = rp1[k] - 1.0
    return elem, rst


def probe_weights(mesh: Mesh, ref: RefElement, pts: np.ndarray):
    elem, rst = locate(mesh, pts)
    return elem, ref.lagrange(rst)


def probe(q: np.ndarray, elem: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Field values [n_probes, 6] (Ex..Hz)."""
    return np.einsum("pj,pcj->pc", W, q[elem, 0:6])
