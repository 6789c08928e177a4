"""Assemble and run a whole simulation in the oracle (FP64).

Inputs (mesh, cubature rule, recipe dict) come from the caller; see
``paper_2006_02551_amd.inputs`` for the recipes.  The time step follows the
recipe's rule dt = cfl / ((N+1)^2 max_{k,f} Fscale_{k,f}).
"""
from __future__ import annotations

import numpy as np

from . import lserk
from .brute import BruteOperator
from .ec import ECOperator
from .mesh import Mesh
from .readout import energy, probe, probe_weights
from .refel import RefElement
from .rhs import Operator


class Simulation:
    def __init__(self, cfg: dict, vxyz, etov, rst, w, brute: bool = False, sigma_q=None, scheme: str = "waa",
                 brute_points: int = 9, vertex_id=None, brute_rule=None):
        self.cfg = cfg
        self.ref = RefElement(cfg["N"], rst, w)
        self.mesh = Mesh(vxyz, etov, self.ref, vertex_id=vertex_id)
        scheme = "direct" if brute else scheme
        if scheme == "direct":
            self.op = BruteOperator(self.mesh, self.ref, cfg["pml"], cfg["alpha"], cfg.get("source"),
                                    quad_points=brute_points, rule=brute_rule)
        elif scheme == "ec":
            self.op = ECOperator(self.mesh, self.ref, cfg["pml"], cfg["alpha"], cfg.get("source"))
        else:
            self.op = Operator(self.mesh, self.ref, cfg["pml"], cfg["alpha"], cfg.get("source"), sigma_q=sigma_q)
        self.dt = float(cfg["cfl"]) / ((cfg["N"] + 1) ** 2 * np.max(self.mesh.Fscale))
        self.t = 0.0
        self.q = np.zeros((self.mesh.K, 12, self.ref.Np))
        self.probe_elem = None
        if cfg.get("probes") is not None:
            self.probe_elem, self.probe_W = probe_weights(self.mesh, self.ref, np.asarray(cfg["probes"]))

    def set_state(self, q):
        q = np.array(q, dtype=np.float64, copy=True)
        q[~self.op.is_pml, 6:12] = 0.0
        self.q = q

    def rhs(self, q, t):
        return self.op.rhs(q, t)

    def run(self, nsteps: int, dt: float | None = None, record_probes: bool = False):
        dt = self.dt if dt is None else dt
        rows = []
        for _ in range(nsteps):
            self.q = lserk.step(self.rhs, self.q, self.t, dt)
            self.t += dt
            if record_probes and self.probe_elem is not None:
                rows.append(probe(self.q, self.probe_elem, self.probe_W))
        return np.asarray(rows) if record_probes else None

    def energy(self) -> float:
        return energy(self.mesh, self.ref, self.q)
