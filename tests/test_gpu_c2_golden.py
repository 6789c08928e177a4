"""The 48,000-tet N = 3 dipole workload over its full 1,000 steps against the FP64 oracle (GPU).

The oracle run is stored in tests/golden/c2_oracle_1000.npz (written by tests/golden/make_c2_golden.py,
which calls only the oracle and the seeded inputs): probe rows after every step, energies and the states of
a fixed element sample after steps 100, 500 and 1,000.  The library steps the same workload in the launch
configuration the benchmark times; FP64 must agree to 1e-12 and FP32 to 1e-5: the relative L2 error of E,H
over the sample; the auxiliary fields' L2 error relative to the larger of their norm and the E,H norm (before
the radiation reaches the layer they hold only rounding-level values); probe rows relative to their largest
value; energies relative.
"""
import os
import sys

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_1000.npz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_c2_1000_steps_against_oracle(precision, tol):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg
    g = np.load(GOLDEN)
    cfg = inputs.config("c2")
    vx, ev = inputs.mesh_for(cfg)
    sim = wdg.Simulation(vx, ev, cfg["N"], inputs.load_rule(cfg["cub_degree"]), cfg["pml"], cfg["alpha"], precision)
    d = sim.dims
    sim.set_dipole(cfg["source"])
    sim.set_probes(np.asarray(cfg["probes"]), cfg["steps"] + 1)
    sim.set_fields(np.zeros((d.K, 12, d.Np)))
    dt = float(g["dt"])
    assert abs(dt - cfg["cfl"] * d.dt_unit) <= 1e-14 * dt
    elems = g["elems"]
    done = 0
    for n, want_e in zip(g["energy_steps"], g["energy"]):
        _say(f"c2 golden: precision {precision}, stepping to {n}")
        sim.step(dt, int(n) - done)
        done = int(n)
        q = sim.get_fields()[elems]
        ref = g[f"q{n}"]
        eh = _rel(q[:, :6], ref[:, :6])
        naux, neh = np.linalg.norm(ref[:, 6:]), np.linalg.norm(ref[:, :6])
        daux = float(np.linalg.norm(q[:, 6:] - ref[:, 6:]))
        de = abs(sim.energy() - want_e) / want_e
        _say(f"  step {n}: relative L2 error E,H {eh:.3e}; auxiliary {daux / max(naux, 1e-300):.3e} of its norm "
             f"({naux:.2e}), {daux / neh:.3e} of the E,H norm; energy {de:.3e}")
        assert eh <= tol and daux <= tol * max(naux, neh) and de <= tol
    rows = sim.probe_read(cfg["steps"] + 1)
    perr = np.max(np.abs(rows - g["probes"])) / np.max(np.abs(g["probes"]))
    _say(f"  probe rows ({rows.shape[0]} steps x 8 probes x 6): max error {perr:.3e} of the largest value")
    assert rows.shape == g["probes"].shape
    assert perr <= tol
    assert np.max(np.abs(ref[:, 6:])) > 0  # the radiation has reached the layer
