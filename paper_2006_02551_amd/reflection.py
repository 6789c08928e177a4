"""Plane-wave reflection from the absorbing layer (the normal-incidence study of Sec. III).

A plane pulse travels along a column that is periodic in x and y (so it stays plane), crosses the PML
interface, is absorbed on its way to the PEC wall and back, and what returns is recorded at a probe
between the initial pulse and the layer.  A plane wave along +z has E_x = H_y and one along -z has
E_x = -H_y, so (E_x + H_y)/2 and (E_x - H_y)/2 at the probe separate the incident pulse (with its
dispersive wake, which also runs along +z) from what comes back.  The reflection is the largest
|E_x - H_y|/2 after the incident pulse has passed, relative to the incident peak of |E_x + H_y|/2;
for small sigma_max it is the wall's echo
attenuated twice through the layer (about exp(-2 sigma_max L / (p + 1)) for the profile
sigma_max (d/L)^p), for large sigma_max the discretisation's own reflection from the steep profile
takes over, and the best sigma_max lies between.  The scan runs the weight-adjusted scheme, the direct
scheme with stored matrices and element-constant coefficients on the same mesh.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs, wdg

SCHEMES = {"waa": wdg.WDG_PML_WAA, "direct": wdg.WDG_PML_DIRECT, "constant": wdg.WDG_PML_CONSTANT}


class Column:
    """The recipe's column at order N (cubature of degree 2N) in one library context."""

    def __init__(self, cfg: dict, N: int | None = None, precision=wdg.WDG_FP64):
        self.cfg = cfg
        self.N = int(N if N is not None else cfg["N"])
        self.vx, self.ev, self.vid = inputs.column_for(cfg)
        self.rule = inputs.load_rule(2 * self.N)
        self.precision = precision

    def run(self, sigma_max: float, scheme: str = "waa", order: float | None = None) -> dict:
        cfg = self.cfg
        pml = dict(cfg["pml"], sigma_max=[0.0, 0.0, float(sigma_max)])
        if order is not None:
            pml["order"] = float(order)
        sim = wdg.Simulation(self.vx, self.ev, self.N, self.rule, pml, cfg["alpha"], self.precision,
                             vertex_id=self.vid)
        if scheme != "waa":
            sim.set_pml_scheme(SCHEMES[scheme], inputs.product_rule(self.N + 4) if scheme == "direct" else None)
        dt0 = cfg["cfl"] * sim.dims.dt_unit
        nsteps = int(math.ceil(cfg["t_end"] / dt0))
        dt = cfg["t_end"] / nsteps
        sim.set_fields(inputs.plane_pulse_fields(cfg, sim.node_coords()))
        sim.set_probes([cfg["probe"]], nsteps + 1)
        sim.step(dt, nsteps)
        rows = sim.probe_read(nsteps + 1)[:, 0, :]
        ex, hy = rows[:, 0], rows[:, 4]
        t = dt * np.arange(1, len(ex) + 1)
        fwd, back = 0.5 * (ex + hy), 0.5 * (ex - hy)
        early = np.abs(fwd[t <= cfg["t_split"]]).max()
        late = np.abs(back[t > cfg["t_split"]]).max()
        r = late / early
        del sim
        return {"sigma_max": float(sigma_max), "scheme": scheme, "N": self.N, "steps": nsteps, "dt": dt,
                "incident": float(early), "reflected": float(late), "R": float(r),
                "R_dB": float(20.0 * math.log10(r)), "t": t, "ex": ex, "hy": hy}


def scan(cfg: dict, N: int, schemes=("waa", "direct", "constant"), sigmas=None, precision=wdg.WDG_FP64,
         report=None) -> dict:
    """R in dB per scheme over the recipe's sigma_max list: {scheme: [(sigma_max, R_dB), ...]}.
    report(result) is called after every run."""
    col = Column(cfg, N, precision)
    sigmas = cfg["scan"]["sigma_max"] if sigmas is None else sigmas
    out = {}
    for s in schemes:
        out[s] = []
        for sg in sigmas:
            r = col.run(sg, s)
            out[s].append((sg, r["R_dB"]))
            if report is not None:
                report(r)
    return out
