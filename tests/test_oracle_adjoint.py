"""Pins of the oracle's discrete adjoint and shell-energy gradient (CPU).

The adjoint is checked against the forward operator it transposes (dot-product
identities in the energy inner product), the eq. (9) derivatives against
finite differences of oracle.pml.tensors, and the full gradient against central
finite differences of the loss itself.
"""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle.mesh import Mesh
from oracle.pml import sigma_kappa, tensors
from oracle.refel import RefElement
from oracle.rhs import Operator
from paper_2006_02551_amd import inputs

PML = {"lo": [-0.4] * 3, "hi": [0.4] * 3, "L": [0.6] * 3, "sigma_max": [20.0, 14.0, 26.0], "order": 3.0,
       "kappa_max": 1.0}
SHELL = {"outer_lo": [-0.4] * 3, "outer_hi": [0.4] * 3, "inner_lo": [-0.2] * 3, "inner_hi": [0.2] * 3}


def _setup(N, n, rules, pml=PML, alpha=1.0, pert=0.1, seed=3, deg=None):
    ref = RefElement(N, *rules(deg or 2 * N))
    vx, ev = inputs.kuhn_box(n, -1.0, 1.0, pert, seed=seed)
    mesh = Mesh(vx, ev, ref)
    return Operator(mesh, ref, pml, alpha=alpha)


def _random_state(op, rng):
    q = rng.standard_normal((op.mesh.K, 12, op.ref.Np))
    q[~op.is_pml, 6:] = 0.0
    return q


@pytest.mark.parametrize("N,alpha", [(1, 1.0), (2, 1.0), (2, 0.0), (3, 1.0)])
def test_operator_adjoint_dot_product(N, alpha, rules):
    op = _setup(N, 3, rules, alpha=alpha)
    assert 0 < len(op.pml_elems) < op.mesh.K
    adj = A.Adjoint(op)
    rng = np.random.default_rng(N)
    x, y = _random_state(op, rng), _random_state(op, rng)
    lhs = A.inner_m(op, y, op.rhs(x, 0.0))
    rhs = A.inner_m(op, adj.apply(y), x)
    scale = np.sqrt(A.inner_m(op, y, y) * A.inner_m(op, op.rhs(x, 0.0), op.rhs(x, 0.0)))
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


def test_operator_adjoint_all_pml_and_no_pml(rules):
    rng = np.random.default_rng(7)
    for pml in ({"lo": [0.0] * 3, "hi": [0.0] * 3, "L": [1.0] * 3, "sigma_max": [5.0, 7.0, 9.0], "order": 2.0},
                None):
        op = _setup(2, 2, rules, pml=pml)
        adj = A.Adjoint(op)
        x, y = _random_state(op, rng), _random_state(op, rng)
        lhs = A.inner_m(op, y, op.rhs(x, 0.0))
        rhs = A.inner_m(op, adj.apply(y), x)
        scale = np.sqrt(A.inner_m(op, y, y) * A.inner_m(op, op.rhs(x, 0.0), op.rhs(x, 0.0)))
        assert abs(lhs - rhs) <= 1e-13 * scale


def test_step_adjoint_dot_product(rules):
    op = _setup(2, 3, rules)
    adj = A.Adjoint(op)
    rng = np.random.default_rng(11)
    x, lam = _random_state(op, rng), _random_state(op, rng)
    dt = 0.5 / (9 * np.max(op.mesh.Fscale))
    phix, stages = A.forward_stages(op, x, 0.0, dt)
    back = A.adjoint_step(adj, lam, stages, dt)
    lhs, rhs = A.inner_m(op, lam, phix), A.inner_m(op, back, x)
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(A.inner_m(op, lam, lam) * A.inner_m(op, x, x))


def test_tensor_derivatives_match_finite_differences():
    rng = np.random.default_rng(2)
    sigma = rng.uniform(0.0, 30.0, (40, 3))
    for kappa in (np.ones((40, 3)), rng.uniform(1.0, 3.0, (40, 3))):
        db, dc, dd = A.tensor_derivatives(sigma, kappa)
        h = 1e-5
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            _, bp, cp, dp, _ = tensors(sigma + e, kappa)
            _, bm, cm, dm, _ = tensors(sigma - e, kappa)
            # b and d are linear and c quadratic in sigma: central differences are exact up to rounding
            assert np.allclose((bp - bm) / (2 * h), db[..., a], rtol=1e-7, atol=1e-8)
            assert np.allclose((cp - cm) / (2 * h), dc[..., a], rtol=1e-7, atol=1e-6)
            assert np.allclose((dp - dm) / (2 * h), dd[..., a], rtol=1e-7, atol=1e-8)


def test_shell_gradient_is_exact_for_the_quadratic_energy(rules):
    op = _setup(2, 3, rules)
    chi = A.shell_weights(op, SHELL)
    assert 0 < chi.sum() < chi.size
    rng = np.random.default_rng(5)
    q, dq = _random_state(op, rng), _random_state(op, rng)
    g = A.shell_gradient(op, chi, q)
    fd = (A.shell_energy(op, chi, q + dq) - A.shell_energy(op, chi, q - dq)) / 2.0
    assert abs(A.inner_m(op, g, dq) - fd) <= 1e-12 * abs(fd)


def test_profile_derivatives_match_finite_differences():
    rng = np.random.default_rng(9)
    x = rng.uniform(-1.0, 1.0, (200, 3))
    d = A.profile_derivatives(x, PML)
    base = np.asarray(PML["sigma_max"], float)
    h = 1e-6
    for t in range(7):
        pp, pm = dict(PML), dict(PML)
        if t < 3:
            for pr, sgn in ((pp, 1), (pm, -1)):
                sm = base.copy()
                sm[t] += sgn * h
                pr["sigma_max"] = list(sm)
        elif t < 6:
            Lp, Lm = np.asarray(PML["L"], float).copy(), np.asarray(PML["L"], float).copy()
            Lp[t - 3] += h
            Lm[t - 3] -= h
            pp, pm = A.moved_interface(PML, Lp), A.moved_interface(PML, Lm)
        else:
            pp["order"] = PML["order"] + h
            pm["order"] = PML["order"] - h
        fd = (sigma_kappa(x, pp)[0] - sigma_kappa(x, pm)[0]) / (2 * h)
        assert np.allclose(fd, d[..., t], rtol=1e-6, atol=1e-7), t


def _loss_setup(rules):
    op = _setup(2, 3, rules, deg=4)
    assert 0 < len(op.pml_elems) < op.mesh.K
    rng = np.random.default_rng(1)
    cfg = inputs.config("c1", **{"init.width": 0.35})
    q0 = inputs.gaussian_fields(cfg, op.mesh.x)
    q0[:, 0:6] += 0.1 * rng.standard_normal((op.mesh.K, 6, op.ref.Np))
    q0[op.is_pml, 6:] = 0.05 * rng.standard_normal((len(op.pml_elems), 6, op.ref.Np))
    dt = 0.75 / (9 * np.max(op.mesh.Fscale))
    return op, q0, dt


def test_sigma_gradient_matches_finite_differences(rules):
    op, q0, dt = _loss_setup(rules)
    nsteps = 6
    J, g, _ = A.loss_and_gradient(op, q0, 0.0, dt, nsteps, SHELL)
    assert np.isclose(J, A.loss(op, q0, 0.0, dt, nsteps, SHELL), rtol=1e-13)
    rounding = 100 * np.finfo(float).eps * abs(J)
    rng = np.random.default_rng(4)
    # the largest entries and a few random ones
    flat = np.argsort(np.abs(g).ravel())[::-1][:3].tolist() + rng.choice(g.size, 3, replace=False).tolist()
    for idx in flat:
        k, qn, a = np.unravel_index(idx, g.shape)
        h = 1e-6 * max(1.0, abs(op.sigma[op.pml_elems[k], qn, a]))
        vals = []
        for sgn in (1.0, -1.0):
            s = op.sigma.copy()
            s[op.pml_elems[k], qn, a] += sgn * h
            o2 = Operator(op.mesh, op.ref, None, alpha=op.alpha, sigma_q=s)
            assert np.array_equal(o2.pml_elems, op.pml_elems)
            vals.append(A.loss(o2, q0, 0.0, dt, nsteps, SHELL))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k, qn, a]) <= 1e-6 * abs(fd) + rounding / h, (idx, fd, g[k, qn, a], rounding / h)


def test_profile_gradient_matches_finite_differences(rules):
    op, q0, dt = _loss_setup(rules)
    nsteps = 6
    J, g, _ = A.loss_and_gradient(op, q0, 0.0, dt, nsteps, SHELL)
    gp = A.profile_gradient(op, PML, g)
    # central differences: truncation O(h^2) plus rounding ~ eps |J| / h
    rounding = 100 * np.finfo(float).eps * abs(J)
    assert np.all(np.isfinite(gp)) and np.max(np.abs(gp)) > 0
    h = 1e-6
    for t in range(7):
        vals = []
        for sgn in (1.0, -1.0):
            pr = dict(PML)
            if t < 3:
                sm = np.asarray(PML["sigma_max"], float).copy()
                sm[t] += sgn * h
                pr["sigma_max"] = list(sm)
            elif t < 6:
                Ln = np.asarray(PML["L"], float).copy()
                Ln[t - 3] += sgn * h
                pr = A.moved_interface(PML, Ln)
            else:
                pr["order"] = PML["order"] + sgn * h
            o2 = Operator(op.mesh, op.ref, pr, alpha=op.alpha)
            assert np.array_equal(o2.pml_elems, op.pml_elems)
            vals.append(A.loss(o2, q0, 0.0, dt, nsteps, SHELL))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gp[t]) <= 1e-6 * abs(fd) + rounding / h, (t, fd, gp[t], rounding / h)
