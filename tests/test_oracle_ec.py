"""Pins of the element-constant ("EC-paved") oracle and of the conical product rule input."""
import math

import numpy as np
import pytest

from oracle.brute import BruteOperator
from oracle.ec import ECOperator, ec_samples
from oracle.mesh import Mesh
from oracle.pml import sigma_kappa, tensors
from oracle.refel import RefElement
from oracle.rhs import Operator
from paper_2006_02551_amd import inputs

PML = {"lo": [-0.5] * 3, "hi": [0.5] * 3, "L": [0.5] * 3, "sigma_max": [20.0, 14.0, 9.0], "order": 2.0,
       "kappa_max": 2.0}


def _setup(N, n, rules, pert=0.1, seed=3):
    ref = RefElement(N, *rules(2 * N))
    vx, ev = inputs.kuhn_box(n, -1.0, 1.0, pert, seed=seed)
    return ref, Mesh(vx, ev, ref)


def test_product_rule_moments():
    # exact for barycentric monomials up to degree 2n-1: int l1^i l2^j l3^k = 8 i! j! k! / (i+j+k+3)!
    for n in (2, 4, 7):
        rst, w = inputs.product_rule(n)
        assert rst.shape == (n ** 3, 3) and np.all(w > 0)
        lam = np.column_stack([(1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2, (1 + rst[:, 2]) / 2])
        assert np.all(lam > 0) and np.all(lam.sum(axis=1) < 1)  # strictly interior
        D = 2 * n - 1
        for i in range(D + 1):
            for j in range(D + 1 - i):
                for k in range(D + 1 - i - j):
                    exact = 8.0 * math.factorial(i) * math.factorial(j) * math.factorial(k) / math.factorial(i + j + k + 3)
                    got = np.sum(w * lam[:, 0] ** i * lam[:, 1] ** j * lam[:, 2] ** k)
                    assert abs(got - exact) < 1e-14 * max(1.0, exact), (n, i, j, k)
        # one degree too many is not integrated exactly
        got = np.sum(w * lam[:, 2] ** (2 * n))
        assert abs(got - 8.0 * math.factorial(2 * n) / math.factorial(2 * n + 3)) > 1e-12


def test_ec_samples_are_the_farthest_vertex(rules):
    ref, mesh = _setup(2, 4, rules)
    sig, kap = ec_samples(mesh.x, PML)
    # straight-sided elements: along each axis the farthest node is a vertex
    verts = mesh.vxyz[mesh.etov]  # [K, 4, 3]
    s_v, k_v = sigma_kappa(verts, PML)
    # (vertex nodes are mapped from the reference element, so they match the vertices to rounding)
    assert np.allclose(sig, s_v.max(axis=1), rtol=1e-13, atol=1e-12)
    assert np.allclose(kap, k_v.max(axis=1), rtol=1e-13, atol=1e-13)
    assert np.any((sig > 0) & (sig < 20.0 * 0.99))  # some elements only partly in the layer
    # a hand-made element: vertices at x = 0.6, 0.7, 0.9 beyond hi = 0.5
    x = np.array([[[0.6, 0.0, 0.0], [0.7, 0.1, 0.0], [0.9, 0.0, 0.1], [0.6, 0.2, 0.2]]])
    s, k = ec_samples(x, PML)
    assert s[0, 0] == pytest.approx(20.0 * (0.4 / 0.5) ** 2, rel=1e-15)
    assert s[0, 1] == 0.0 and s[0, 2] == 0.0
    assert k[0, 0] == pytest.approx(1.0 + (0.4 / 0.5) ** 2, rel=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_ec_equals_waa_with_constant_samples(N, rules):
    ref, mesh = _setup(N, 3, rules)
    ec = ECOperator(mesh, ref, PML)
    # the weight-adjusted operator fed the element constants at every cubature point is exact
    waa = Operator(mesh, ref, PML)
    assert np.array_equal(ec.pml_elems, waa.pml_elems)
    Kp = len(waa.pml_elems)
    sig = np.broadcast_to(ec.ec_sigma[:, None, :], (Kp, ref.Nq, 3))
    kap = np.broadcast_to(ec.ec_kappa[:, None, :], (Kp, ref.Nq, 3))
    waa.a, waa.b, waa.c, waa.d, waa.kap = tensors(sig, kap)
    rng = np.random.default_rng(N)
    q = rng.standard_normal((mesh.K, 12, ref.Np))
    q[~waa.is_pml, 6:] = 0.0
    r1, r2 = ec.rhs(q, 0.0), waa.rhs(q, 0.0)
    assert np.max(np.abs(r1 - r2)) < 1e-11 * np.max(np.abs(r2))
    # and the direct scheme with the same constant weights (exact mass alpha M_k)
    bru = BruteOperator(mesh, ref, PML, quad_points=N + 1)
    a, b, c, d, k = tensors(ec.ec_sigma, ec.ec_kappa)
    Mk = bru.Mk[:, None]
    bru.Ma, bru.Mb, bru.Mc, bru.Md = (x[:, :, None, None] * Mk for x in (a, b, c, d))
    bru.Mik = (1.0 / k)[:, :, None, None] * Mk
    r3 = bru.rhs(q, 0.0)
    assert np.max(np.abs(r1 - r3)) < 1e-10 * np.max(np.abs(r3))


def test_ec_without_conductivity_is_vacuum(rules):
    ref, mesh = _setup(2, 3, rules)
    pml = dict(PML, sigma_max=[0.0, 0.0, 0.0], kappa_max=1.0, lo=[-0.9] * 3, hi=[0.9] * 3)
    pml_on = dict(pml, sigma_max=[1e-300, 0.0, 0.0])  # classifies the layer, coefficients ~ 0
    ec = ECOperator(mesh, ref, pml_on)
    assert len(ec.pml_elems) > 0
    vac = Operator(mesh, ref, None)
    rng = np.random.default_rng(5)
    q = rng.standard_normal((mesh.K, 12, ref.Np))
    q[~ec.is_pml, 6:] = 0.0
    r1, r0 = ec.rhs(q, 0.0), vac.rhs(q, 0.0)
    assert np.max(np.abs(r1[:, :6] - r0[:, :6])) < 1e-12 * np.max(np.abs(r0))
    assert np.array_equal(r1[ec.pml_elems, 6:], q[ec.pml_elems, :6])  # dP = f when kappa = 1, d = 0


def test_direct_oracle_with_the_product_rule_input(rules):
    # the stored-matrix oracle fed the input product rule agrees with its own rule of the same degree on
    # elements whose weights are polynomial (an aligned slab with a linear profile: both rules are exact),
    # and the element subset gives the same rows as the full operator
    N = 2
    ref = RefElement(N, *rules(2 * N))
    vx, ev = inputs.kuhn_box(4, -1.0, 1.0, 0.0, seed=0)
    mesh = Mesh(vx, ev, ref)
    pml = {"lo": [-9.0, -9.0, -0.5], "hi": [9.0, 9.0, 0.5], "L": [1.0, 1.0, 0.5], "sigma_max": [0.0, 0.0, 6.0],
           "order": 1.0, "kappa_max": 1.0}
    a = BruteOperator(mesh, ref, pml, quad_points=6)
    b = BruteOperator(mesh, ref, pml, rule=inputs.product_rule(6))
    rng = np.random.default_rng(8)
    q = rng.standard_normal((mesh.K, 12, ref.Np))
    q[~a.is_pml, 6:] = 0.0
    ra, rb = a.rhs(q, 0.0), b.rhs(q, 0.0)
    assert np.max(np.abs(ra - rb)) < 1e-12 * np.max(np.abs(ra))
    el = a.pml_elems[::7]
    c = BruteOperator(mesh, ref, pml, rule=inputs.product_rule(6), elements=el)
    assert np.max(np.abs(c.rhs(q, 0.0, el=el) - rb[el])) < 1e-14 * np.max(np.abs(ra))
    with pytest.raises(ValueError):
        c.rhs(q, 0.0, el=a.pml_elems[1:2])
