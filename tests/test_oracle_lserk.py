"""Pins of the LSERK4 integrator (CPU): exact rational stability polynomial, stage times, order."""
from fractions import Fraction as Fr

import numpy as np

from oracle import lserk


def _poly_add(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def _poly_scale(p, s):
    return [s * c for c in p]


def _poly_shift(p):  # multiply by z
    return [Fr(0)] + list(p)


def test_stability_polynomial_exact():
    # y' = lambda y with z = lambda dt, exact rational arithmetic:
    # res <- A res + z y ; y <- y + B res
    y = [Fr(1)]
    res = [Fr(0)]
    for i in range(5):
        res = _poly_add(_poly_scale(res, lserk.A_FR[i]), _poly_shift(y))
        y = _poly_add(y, _poly_scale(res, lserk.B_FR[i]))
    # The published 13-digit rationals meet the order conditions to ~1e-25,
    # far below FP64 rounding; the fifth-order term is 1/200.
    expect = [Fr(1), Fr(1), Fr(1, 2), Fr(1, 6), Fr(1, 24), Fr(1, 200)]
    assert len(y) == 6
    for got, want in zip(y, expect):
        assert abs(got - want) < Fr(1, 10 ** 24)


def test_stage_times():
    # for y' = 1 the state entering stage i equals c_i dt exactly
    y, res = Fr(0), Fr(0)
    for i in range(5):
        assert abs(y - lserk.C_FR[i]) < Fr(1, 10 ** 24)
        res = lserk.A_FR[i] * res + 1
        y = y + lserk.B_FR[i] * res
    assert abs(y - 1) < Fr(1, 10 ** 24)


def test_fourth_order():
    lam = -0.7

    def f(y, t):
        return lam * y + np.cos(t)

    def exact(t):
        # y' = lam y + cos t, y(0) = 1
        A = (lam * 0 + 1)  # particular solution coefficients
        c1 = -lam / (lam ** 2 + 1)
        c2 = 1 / (lam ** 2 + 1)
        return (1 - c1) * np.exp(lam * t) + c1 * np.cos(t) + c2 * np.sin(t) + 0 * A

    errs = []
    for n in (10, 20, 40):
        dt = 2.0 / n
        y = np.array(1.0)
        t = 0.0
        for _ in range(n):
            y = lserk.step(f, y, t, dt)
            t += dt
        errs.append(abs(float(y) - exact(2.0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 4.0) < 0.25), rates


def test_cavity_energy_under_the_dt_rule_and_blow_up_beyond_it():
    """A vacuum PEC cavity with the upwind flux: the semi-discrete energy does not grow, so LSERK4 at the recipes'
    dt rule (inside its stability region) keeps the energy at or below its start and the upwind flux dissipates
    some of it; fifty times that step leaves the region and the energy grows until it is no longer finite, the
    condition the library's energy readout reports as WDG_ENONFINITE."""
    from oracle.run import Simulation
    from paper_2006_02551_amd import inputs

    cfg = inputs.config("c1", **{"mesh.n": 2, "mesh.perturb": 0.1, "pml.lo": [-1.0] * 3, "pml.hi": [1.0] * 3})
    vx, ev = inputs.mesh_for(cfg)
    rst, w = inputs.load_rule(cfg["cub_degree"])
    q0 = np.random.default_rng(7).standard_normal((ev.shape[0], 12, (cfg["N"] + 1) * (cfg["N"] + 2) * (cfg["N"] + 3) // 6))
    sim = Simulation(cfg, vx, ev, rst, w)
    assert not sim.op.is_pml.any()
    sim.set_state(q0)
    e = [sim.energy()]
    for _ in range(30):
        sim.run(1)
        e.append(sim.energy())
    assert max(e) <= e[0] * (1 + 1e-12)
    assert e[-1] < 0.9 * e[0]

    big = Simulation(cfg, vx, ev, rst, w)
    big.set_state(q0)
    with np.errstate(over="ignore", invalid="ignore"):
        big.run(3, dt=50 * sim.dt)
        assert big.energy() > 1e6 * e[0]
        for _ in range(200):
            big.run(1, dt=50 * sim.dt)
            if not np.isfinite(big.energy()):
                break
        assert not np.isfinite(big.energy())
