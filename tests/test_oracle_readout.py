"""Pins of the oracle's energy and probe readouts (CPU)."""
import numpy as np

from oracle.mesh import Mesh
from oracle.readout import energy, probe, probe_weights
from oracle.refel import RefElement
from paper_2006_02551_amd import inputs


def _mesh(rules, N=3):
    ref = RefElement(N, *rules(2 * N))
    vx, ev = inputs.kuhn_box(3, -1.5, 1.5, 0.1, seed=2)
    return ref, Mesh(vx, ev, ref)


def test_energy_of_constant_field(rules):
    ref, mesh = _mesh(rules)
    q = np.zeros((mesh.K, 12, ref.Np))
    q[:, 0] = 2.0
    q[:, 4] = -1.0
    # 1/2 (|E|^2 + |H|^2) * volume = 1/2 * 5 * 27
    assert abs(energy(mesh, ref, q) - 0.5 * 5.0 * 27.0) < 1e-11


def test_probes_reproduce_polynomials(rules):
    ref, mesh = _mesh(rules)
    x = mesh.x
    q = np.zeros((mesh.K, 12, ref.Np))
    q[:, 1] = x[..., 0] ** 3 - 2 * x[..., 1] * x[..., 2] + 0.5
    q[:, 5] = x[..., 2] ** 2
    pts = np.array([[0.5, 0.5, 0.5], [-0.5, 0.37, 0.11], [1.2, -1.3, 0.7]])
    elem, W = probe_weights(mesh, ref, pts)
    vals = probe(q, elem, W)
    assert np.allclose(vals[:, 1], pts[:, 0] ** 3 - 2 * pts[:, 1] * pts[:, 2] + 0.5, atol=1e-12)
    assert np.allclose(vals[:, 5], pts[:, 2] ** 2, atol=1e-12)
    assert np.allclose(vals[:, [0, 2, 3, 4]], 0.0)
