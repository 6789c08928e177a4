"""Pins of the oracle's reference element against closed forms (CPU)."""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.refel import FACE_VERTS, REF_VERTS, RefElement, equispaced_nodes
from tests import exact


_RULES = os.listdir(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                 "paper_2006_02551_amd", "inputs", "cubature"))
ORDERS = [N for N in (1, 2, 3, 4) if f"tet_deg{2 * N}.txt" in _RULES]


@pytest.fixture(scope="module", params=ORDERS)
def ref(request, rules):
    N = request.param
    rst, w = rules(2 * N)
    return RefElement(N, rst, w)


def test_counts(ref):
    N = ref.N
    assert ref.Np == (N + 1) * (N + 2) * (N + 3) // 6
    assert all(len(f) == (N + 1) * (N + 2) // 2 for f in ref.fmask)
    assert equispaced_nodes(N).shape == (ref.Np, 3)


def test_derivatives_exact_on_polynomials(ref):
    X = ref.nodes
    for (a, b, c) in exact.monomials(ref.N):
        p = X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c
        dr = a * X[:, 0] ** max(a - 1, 0) * X[:, 1] ** b * X[:, 2] ** c if a else 0 * p
        ds = b * X[:, 0] ** a * X[:, 1] ** max(b - 1, 0) * X[:, 2] ** c if b else 0 * p
        dt = c * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** max(c - 1, 0) if c else 0 * p
        assert np.max(np.abs(ref.Dr @ p - dr)) < 1e-11
        assert np.max(np.abs(ref.Ds @ p - ds)) < 1e-11
        assert np.max(np.abs(ref.Dt @ p - dt)) < 1e-11


def test_mass_matrix_integrates_products(ref):
    X = ref.nodes
    assert np.allclose(ref.M, ref.M.T, atol=1e-15)
    assert np.all(np.linalg.eigvalsh(ref.M) > 0)
    assert abs(np.sum(ref.M) - 4.0 / 3.0) < 1e-13
    mons = exact.monomials(ref.N)
    for e1 in mons[:: max(1, len(mons) // 6)]:
        for e2 in mons[:: max(1, len(mons) // 5)]:
            p = exact.eval_poly(exact.monomial(*e1), X)
            q = exact.eval_poly(exact.monomial(*e2), X)
            ex = float(exact.integrate(exact.poly_mul(exact.monomial(*e1), exact.monomial(*e2)),
                                       exact.REF_TET, exact.REF_VOL))
            assert abs(p @ ref.M @ q - ex) < 1e-13


def test_lift_reproduces_face_integrals(ref):
    # 1^T M LIFT_f g = int_{face f} g over the reference face measure (area 2)
    X = ref.nodes
    ones = np.ones(ref.Np)
    for f, tri in enumerate(FACE_VERTS):
        verts = [tuple(REF_VERTS[i]) for i in tri]
        blk = ref.LIFT[:, f * ref.Nfp:(f + 1) * ref.Nfp]
        for e in exact.monomials(ref.N):
            g = exact.eval_poly(exact.monomial(*e), X[ref.fmask[f]])
            ex = float(exact.integrate(exact.monomial(*e), verts, Fr(2)))
            assert abs(ones @ ref.M @ blk @ g - ex) < 1e-12, (f, e)
        # the other faces' columns do not leak into face f's integral of a face polynomial
        assert np.max(np.abs(blk)) > 0


def test_vq_interpolates_and_pq_left_inverse(ref):
    X = ref.nodes
    for e in exact.monomials(ref.N):
        p = exact.eval_poly(exact.monomial(*e), X)
        pq = exact.eval_poly(exact.monomial(*e), ref.rq)
        assert np.max(np.abs(ref.Vq @ p - pq)) < 1e-12
    # P_q V_q = I when the rule is exact to degree 2N (eq. (21) with alpha = 1)
    assert np.max(np.abs(ref.Pq @ ref.Vq - np.eye(ref.Np))) < 1e-12


def test_waa_exact_for_constant_weight(ref):
    # eq. (21) with alpha constant in the element: P_q alpha^{-1} V_q M_k^{-1} = (alpha M_k)^{-1}
    alpha = 3.7
    waa = ref.Pq @ np.diag(np.full(ref.Nq, 1.0 / alpha)) @ ref.Vq @ ref.Minv
    assert np.max(np.abs(waa - np.linalg.inv(alpha * ref.M))) < 1e-11


def test_weighted_mass_by_cubature_eq19(ref):
    # eq. (19)-(20): V_q^T W diag(alpha) V_q equals the exact weighted mass matrix
    # for a polynomial weight whose product with l_i l_j stays within the rule degree.
    X = ref.nodes
    deg_rule = 2 * ref.N
    wpoly = {(0, 0, 0): Fr(2), (1, 0, 0): Fr(1, 3)} if deg_rule >= 2 * ref.N + 1 else {(0, 0, 0): Fr(5, 2)}
    alpha_q = exact.eval_poly(wpoly, ref.rq)
    Mw = ref.Vq.T @ np.diag(ref.wq * alpha_q) @ ref.Vq
    mons = exact.monomials(ref.N)
    for e1 in mons[:4]:
        for e2 in mons[-3:]:
            p = exact.eval_poly(exact.monomial(*e1), X)
            q = exact.eval_poly(exact.monomial(*e2), X)
            ex = float(exact.integrate(exact.poly_mul(wpoly, exact.poly_mul(exact.monomial(*e1), exact.monomial(*e2))),
                                       exact.REF_TET, exact.REF_VOL))
            assert abs(p @ Mw @ q - ex) < 1e-12
