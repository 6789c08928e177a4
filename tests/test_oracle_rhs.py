"""Pins of the oracle's semi-discrete operator, eqs. (10)-(17) and (26)-(29) (CPU)."""
import numpy as np
import pytest

from oracle import lserk
from oracle.brute import BruteOperator
from oracle.mesh import Mesh
from oracle.readout import energy
from oracle.refel import RefElement
from oracle.rhs import Operator
from paper_2006_02551_amd import inputs


def _setup(N, n, rules, lo=-1.0, hi=1.0, pert=0.0, deg=None, seed=0):
    ref = RefElement(N, *rules(deg or 2 * N))
    vx, ev = inputs.kuhn_box(n, lo, hi, pert, seed=seed)
    return ref, Mesh(vx, ev, ref)


def _energy_rate(mesh, ref, q, dq):
    return float(np.sum(mesh.J * np.einsum("kci,ij,kcj->k", q[:, 0:6], ref.M, dq[:, 0:6])))


@pytest.mark.parametrize("N", [1, 2, 3])
def test_central_flux_conserves_and_upwind_dissipates(N, rules):
    ref, mesh = _setup(N, 2, rules, pert=0.15, seed=4)
    rng = np.random.default_rng(N)
    q = np.zeros((mesh.K, 12, ref.Np))
    q[:, 0:6] = rng.standard_normal((mesh.K, 6, ref.Np))
    e = energy(mesh, ref, q)
    central = Operator(mesh, ref, None, alpha=0.0)
    rate0 = _energy_rate(mesh, ref, q, central.rhs(q, 0.0))
    assert abs(rate0) < 1e-11 * e
    upwind = Operator(mesh, ref, None, alpha=1.0)
    rate1 = _energy_rate(mesh, ref, q, upwind.rhs(q, 0.0))
    assert rate1 < -1e-3 * e


def test_energy_nonincreasing_in_time(rules):
    ref, mesh = _setup(2, 2, rules)
    op = Operator(mesh, ref, None, alpha=1.0)
    cfg = inputs.config("c1")
    q = inputs.gaussian_fields(cfg, mesh.x)
    dt = 0.75 / (9 * np.max(mesh.Fscale))
    e_prev = energy(mesh, ref, q)
    for _ in range(30):
        q = lserk.step(op.rhs, q, 0.0, dt)
        e = energy(mesh, ref, q)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e


def _cavity(N, n, rules, T=0.25, sigma=None):
    ref, mesh = _setup(N, n, rules, lo=0.0, hi=1.0)
    sq = None if sigma is None else np.full((mesh.K, ref.Nq, 3), sigma)
    op = Operator(mesh, ref, None, alpha=1.0, sigma_q=sq)
    w = np.pi * np.sqrt(2.0)
    x, y = mesh.x[..., 0], mesh.x[..., 1]
    q = np.zeros((mesh.K, 12, ref.Np))
    q[:, 2] = np.sin(np.pi * x) * np.sin(np.pi * y)
    nsteps = int(np.ceil(T / (0.5 / ((N + 1) ** 2 * np.max(mesh.Fscale)))))
    dt = T / nsteps
    t = 0.0
    for _ in range(nsteps):
        q = lserk.step(op.rhs, q, t, dt)
        t += dt
    ex = np.zeros_like(q)
    ex[:, 2] = np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(w * T)
    ex[:, 3] = -(np.pi / w) * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(w * T)
    ex[:, 4] = (np.pi / w) * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(w * T)
    return mesh, ref, op, q, ex


@pytest.mark.parametrize("N", [2, 3])
def test_pec_cavity_mode_converges(N, rules):
    errs = []
    for n in (2, 4):
        mesh, ref, _, q, ex = _cavity(N, n, rules)
        d = q - ex
        errs.append(np.sqrt(2 * energy(mesh, ref, d)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 1 - 0.3, (errs, rate)


def test_uniform_sigma_is_exponential_decay(rules):
    # sigma_x = sigma_y = sigma_z = s, kappa = 1: b = s, c = 0, so the fields are
    # e^{-s t} times the lossless fields (up to the LSERK error of the two runs).
    s = 1.3
    T = 0.25
    mesh, ref, op, q_loss, _ = _cavity(2, 2, rules, T=T, sigma=s)
    assert np.allclose(op.b, s) and np.allclose(op.c, 0.0) and np.allclose(op.d, s)
    _, _, _, q_free, _ = _cavity(2, 2, rules, T=T)
    rel = np.linalg.norm(q_loss[:, 0:6] - np.exp(-s * T) * q_free[:, 0:6]) / np.linalg.norm(q_free[:, 0:6])
    assert rel < 1e-7


def test_local_pml_operator(rules):
    # zero curl: d/dt (f, P) = [[-b, -c], [1/kappa, -d]] (f, P) for constant coefficients
    ref, mesh = _setup(2, 1, rules)
    sig = np.array([0.7, 1.9, 3.1])
    kap = np.array([1.5, 1.2, 2.0])
    op = Operator(mesh, ref, None, sigma_q=np.broadcast_to(sig, (mesh.K, ref.Nq, 3)).copy())
    op.kap = np.broadcast_to(kap, op.kap.shape).copy()
    from oracle.pml import tensors
    a, b, c, d, k = tensors(sig[None], kap[None])
    op.a = np.broadcast_to(a, op.a.shape).copy()
    op.b = np.broadcast_to(b, op.b.shape).copy()
    op.c = np.broadcast_to(c, op.c.shape).copy()
    op.d = np.broadcast_to(d, op.d.shape).copy()
    rng = np.random.default_rng(0)
    f = np.broadcast_to(rng.standard_normal(3)[None, :, None], (mesh.K, 3, ref.Np)).copy()
    P = np.broadcast_to(rng.standard_normal(3)[None, :, None], (mesh.K, 3, ref.Np)).copy()
    R = np.zeros_like(f)
    df, dP = op.pml_update(f, P, R, np.arange(mesh.K))
    a_, b_, c_, d_ = a[0], b[0], c[0], d[0]
    exp_df = (-(b_[:, None] * f[0] + c_[:, None] * P[0]) / a_[:, None])
    exp_dP = f[0] / kap[:, None] - d_[:, None] * P[0]
    assert np.max(np.abs(df - exp_df)) < 1e-12
    assert np.max(np.abs(dP - exp_dP)) < 1e-12
    # z-slab (sigma only along z, kappa = 1): H_z block [[sigma, -sigma^2], [1, -sigma]] is nilpotent
    a, b, c, d, k = tensors(np.array([[0.0, 0.0, 2.0]]), np.ones((1, 3)))
    A = np.array([[-b[0, 2], -c[0, 2]], [1.0, -d[0, 2]]])
    assert np.allclose(A, [[2.0, -4.0], [1.0, -2.0]]) and np.allclose(A @ A, 0.0)


def test_waa_equals_direct_where_exact(rules):
    # kappa step (order 0, kappa_max 2) with constant sigma inside an aligned slab:
    # every coefficient is constant per element, so eq. (18) is exact and the
    # WAA scheme equals the stored-mass scheme to rounding.
    N = 2
    ref, mesh = _setup(N, 4, rules, deg=2 * N + 2)
    pml = {"lo": [-9.0, -9.0, -0.5], "hi": [9.0, 9.0, 0.5], "L": [1.0, 1.0, 0.5],
           "sigma_max": [0.0, 0.0, 6.0], "order": 0.0, "kappa_max": 2.0}
    waa = Operator(mesh, ref, pml)
    bru = BruteOperator(mesh, ref, pml)
    assert np.any(waa.kap != 1.0)
    rng = np.random.default_rng(1)
    q = rng.standard_normal((mesh.K, 12, ref.Np))
    q[~waa.is_pml, 6:] = 0
    r1, r2 = waa.rhs(q, 0.0), bru.rhs(q, 0.0)
    assert np.max(np.abs(r1 - r2)) < 1e-10 * np.max(np.abs(r2))
    # linear sigma, kappa = 1, rule of degree 2N+2: b, c, d, 1/kappa are polynomials of
    # degree <= 2 inside each element of the aligned slab, so eq. (19) is exact too.
    pml1 = dict(pml, order=1.0, kappa_max=1.0)
    waa = Operator(mesh, ref, pml1)
    bru = BruteOperator(mesh, ref, pml1)
    r1, r2 = waa.rhs(q, 0.0), bru.rhs(q, 0.0)
    assert np.max(np.abs(r1 - r2)) < 1e-10 * np.max(np.abs(r2))


def test_waa_error_below_discretisation(rules):
    # General smooth profile with kappa_max = 2: WAA and direct differ, and the
    # difference shrinks under refinement faster than first order.
    N = 2
    diffs = []
    for n in (2, 4):
        ref, mesh = _setup(N, n, rules, deg=2 * N)
        pml = {"lo": [-0.5] * 3, "hi": [0.5] * 3, "L": [0.5] * 3, "sigma_max": [20.0] * 3,
               "order": 2.0, "kappa_max": 2.0}
        waa = Operator(mesh, ref, pml)
        bru = BruteOperator(mesh, ref, pml)
        x = mesh.x
        q = np.zeros((mesh.K, 12, ref.Np))
        q[:, 2] = np.cos(1.3 * x[..., 0]) * np.sin(0.7 * x[..., 1] + 0.2)
        q[:, 4] = np.cos(0.9 * x[..., 2])
        q[waa.is_pml, 8] = np.sin(x[waa.is_pml, :, 1])
        r1, r2 = waa.rhs(q, 0.0), bru.rhs(q, 0.0)
        sel = waa.is_pml
        diffs.append(np.sqrt(np.sum(mesh.J[sel, None, None] * (r1[sel] - r2[sel]) ** 2)))
    assert diffs[1] < diffs[0] / 2.0 ** 1.5, diffs
