"""Write tests/golden/c2_oracle_1000.npz: the FP64 oracle run over the whole 48,000-tet N = 3 workload.

The workload is the dipole-driven cube of the c2 recipe (Sec. III stand-in: 20^3 x 6 perturbed tetrahedra,
N = 3, cubic profile with sigma_max = 30, Gaussian-modulated dipole, 8 probes) stepped 1,000 times with the
five-stage fourth-order low-storage Runge-Kutta scheme.  Stored, all computed by ``oracle/`` from the seeded
inputs of ``paper_2006_02551_amd.inputs`` (nothing from the HIP library):

  dt          the recipe's time step
  probes      [1000, 8, 6] field values at the probes after every step
  energy      energies after steps 100, 500 and 1000 (energy_steps)
  elems       a fixed sample of element indices (user order)
  q100, q500, q1000   the 12-component states of the sampled elements after those steps [n, 12, N_p]

The sample holds every element where the final fields are largest, auxiliary-field elements of the layer
and a seeded random draw, so that the relative error over it is dominated by where the solution lives.

The right-hand side of each stage is evaluated by the oracle's operator on element chunks in forked worker
processes (the oracle's per-element arithmetic, unchanged; the chunks only split the element loop).

Usage: ``python tests/golden/make_c2_golden.py [out.npz] [workers]`` (about an hour with 7 workers).
"""
from __future__ import annotations

import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.pool import ChunkedRHS  # noqa: E402
from oracle.run import Simulation  # noqa: E402
from paper_2006_02551_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_1000.npz")
SAVE_AT = (100, 500, 1000)


def main(out: str = OUT, workers: int = 7) -> None:
    cfg = inputs.config("c2")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    t0 = time.time()
    sim = Simulation(cfg, vx, ev, *rule)
    print(f"setup {time.time() - t0:.1f} s, K = {sim.mesh.K}, K_pml = {len(sim.op.pml_elems)}, dt = {sim.dt!r}",
          flush=True)
    K = sim.mesh.K
    pool = ChunkedRHS(sim.op, sim.q.shape, int(workers))
    sim.rhs = pool
    states, energies, probes = {}, [], []
    t0 = time.time()
    for n in range(1, cfg["steps"] + 1):
        probes.append(sim.run(1, record_probes=True)[0])
        if n in SAVE_AT:
            states[n] = sim.q.copy()
            energies.append(sim.energy())
        if n % 10 == 0:
            print(f"step {n}: t = {sim.t:.6f}, {(time.time() - t0) / n:.2f} s/step", flush=True)
    final = states[SAVE_AT[-1]]
    mag = np.max(np.abs(final), axis=(1, 2))
    rng = np.random.default_rng(2006)
    big = np.argsort(mag)[-192:]
    pml_live = sim.op.pml_elems[np.max(np.abs(final[sim.op.pml_elems, 6:]), axis=(1, 2)) > 0]
    layer = rng.choice(pml_live, min(64, len(pml_live)), replace=False) if len(pml_live) else np.zeros(0, int)
    elems = np.unique(np.concatenate([big, layer, rng.choice(K, 128, replace=False), [0, K - 1]])).astype(np.int64)
    np.savez_compressed(out, dt=np.float64(sim.dt), probes=np.asarray(probes), energy=np.asarray(energies),
                        energy_steps=np.asarray(SAVE_AT), elems=elems,
                        **{f"q{n}": states[n][elems] for n in SAVE_AT})
    pool.close()
    print(f"wrote {out}: {len(elems)} sampled elements, {time.time() - t0:.0f} s stepping", flush=True)


if __name__ == "__main__":
    main(*sys.argv[1:])
