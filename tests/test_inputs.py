"""Pins of the shared inputs: cubature rules and meshes (CPU)."""
import math
import os

import numpy as np
import pytest

from paper_2006_02551_amd import inputs
from paper_2006_02551_amd.inputs.configs import RULE_DIR
from tests import exact

DEGREES = sorted(int(f[7:-4]) for f in os.listdir(RULE_DIR) if f.startswith("tet_deg"))


def _bary_moment(a, b, c, d):
    # int over the reference tet of lam0^a lam1^b lam2^c lam3^d (Dirichlet; volume 4/3)
    return 8.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) * math.factorial(d) / \
        math.factorial(a + b + c + d + 3)


@pytest.mark.parametrize("deg", DEGREES)
def test_rule_exact_positive_interior(deg):
    rst, w = inputs.load_rule(deg)
    assert np.all(w > 0)
    lam = np.column_stack([-(1 + rst.sum(1)) / 2, (1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2, (1 + rst[:, 2]) / 2])
    assert np.all(lam > 0)
    assert abs(w.sum() - 4.0 / 3.0) < 1e-14
    # all four-barycentric monomials of total degree <= deg (a different basis from the fit)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                for d in range(deg + 1 - a - b - c):
                    val = np.sum(w * lam[:, 0] ** a * lam[:, 1] ** b * lam[:, 2] ** c * lam[:, 3] ** d)
                    ex = _bary_moment(a, b, c, d)
                    assert abs(val - ex) <= 1e-14 + 2e-13 * ex, (a, b, c, d, val, ex)


@pytest.mark.parametrize("deg", [d for d in DEGREES if d >= 2])
def test_rule_exact_cartesian_monomials(deg):
    rst, w = inputs.load_rule(deg)
    for e in exact.monomials(deg):
        ex = float(exact.integrate(exact.monomial(*e), exact.REF_TET, exact.REF_VOL))
        val = float(np.sum(w * exact.eval_poly(exact.monomial(*e), rst)))
        assert abs(val - ex) < 1e-13, (e, val, ex)


@pytest.mark.parametrize("n,pert", [(1, 0.0), (3, 0.0), (4, 0.1)])
def test_kuhn_mesh(n, pert):
    vx, ev = inputs.kuhn_box(n, -1.0, 1.0, pert, seed=3)
    assert ev.shape == (6 * n ** 3, 4)
    v = vx[ev]
    vol6 = np.einsum("ki,ki->k", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    assert np.all(vol6 > 0)
    assert abs(vol6.sum() / 6.0 - 8.0) < 1e-12
    # conformity: every face shared by at most two tets, boundary faces = 2 per cube face
    faces = {}
    for k in range(len(ev)):
        for tri in ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)):
            key = tuple(sorted(ev[k, list(tri)]))
            faces[key] = faces.get(key, 0) + 1
    counts = np.array(list(faces.values()))
    assert counts.max() == 2
    assert np.sum(counts == 1) == 12 * n * n


def test_perturbation_keeps_boundary_and_is_seeded():
    a, _ = inputs.kuhn_box(4, -1.5, 1.5, 0.1, seed=0)
    b, _ = inputs.kuhn_box(4, -1.5, 1.5, 0.1, seed=0)
    c, _ = inputs.kuhn_box(4, -1.5, 1.5, 0.0)
    assert np.array_equal(a, b)
    onb = np.any(np.isclose(np.abs(c), 1.5), axis=1)
    assert np.array_equal(a[onb], c[onb])
    h = 3.0 / 4
    assert np.max(np.abs(a - c)) <= 0.1 * h + 1e-15
    assert np.max(np.abs(a - c)) > 0.05 * h
