"""Independent simulations in one library context (the batching form).

The meshes of a batch are concatenated with disjoint vertex sets (no face is
shared, so no flux couples them) into one context: every stage of every
simulation runs in one launch.  Each simulation keeps its own absorbing-layer
profile (wdg_set_sigma_profile) and its own stable time step (a per-element
factor on dt, wdg_set_dt_scale, with the library stepped at dt = 1), so a
simulation in a batch reproduces its standalone run bit for bit.

With group_mb set, every simulation starts at an element-block boundary (WDG_ALIGN_COMPONENTS) and runs of
consecutive simulations whose fields and setup data fit in about group_mb megabytes form step groups: a
captured pair of steps then runs both steps of one group before the next group, so that a group's data stay
in the last-level cache over its ten stages (wdg_set_step_groups).
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs, wdg


class Batch:
    def __init__(self, cfg: dict, precision=wdg.WDG_FP32, recipe=None, group_mb=None):
        self.cfg = cfg
        self.recipe = recipe if recipe is not None else inputs.batch_recipe(cfg["batch"])
        self.meshes = inputs.batch_meshes(cfg, self.recipe)
        vx, ev, self.group, self.offsets = inputs.concat_meshes(self.meshes)
        self.rule = inputs.load_rule(cfg["cub_degree"])
        # any positive profile classifies the elements of the layer the same way
        pml = dict(cfg["pml"], sigma_max=[1.0, 1.0, 1.0], order=2.0)
        flags = wdg.WDG_ALIGN_COMPONENTS if group_mb else 0
        self.sim = wdg.Simulation(vx, ev, cfg["N"], self.rule, pml, cfg["alpha"], precision, flags=flags)
        self.sim.set_sigma_profile(self.group, [[r["sigma_max"]] * 3 for r in self.recipe],
                                   [r["order"] for r in self.recipe])
        fs = self.sim.element_info()["Fscale"].max(axis=1)
        N = cfg["N"]
        self.dt = np.array([cfg["cfl"] / ((N + 1) ** 2 * fs[a:b].max())
                            for a, b in zip(self.offsets[:-1], self.offsets[1:])])
        self.sim.set_dt_scale(self.dt[self.group])
        self.K = int(self.offsets[-1])
        self.step_groups = None
        if group_mb:
            d = self.sim.dims
            word = 8 if precision == wdg.WDG_FP64 else 4
            # bytes per element: three state buffers (fields, auxiliary fields), sigma, geometry, neighbour map
            per_elem = 3 * 12 * d.Np * word + 3 * d.Nq * word + 25 * word + 4 * d.Nfp * 4
            sizes = np.diff(self.offsets) * per_elem
            sim_group, g, acc = [], 0, 0.0
            for sz in sizes:
                if acc > 0 and acc + sz > group_mb * 1e6:
                    g, acc = g + 1, 0.0
                sim_group.append(g)
                acc += sz
            self.step_groups = np.asarray(sim_group, dtype=np.int32)
            self.sim.set_step_groups(self.step_groups[self.group])
        # captured stepping needs a stream other than the null stream; eager steps use it too so that
        # the two never overlap (reading or writing the fields synchronises the device)
        self.stream = torch.cuda.Stream()

    def initial_fields(self):
        return inputs.gaussian_fields(self.cfg, self.sim.node_coords())

    def set_fields(self, q):
        self.sim.set_fields(q)

    def step(self, nsteps, graph=True, stream=None):
        stream = self.stream if stream is None else stream
        if graph:
            self.sim.step_graph(1.0, nsteps, stream)
        else:
            self.sim.step(1.0, nsteps, stream)

    def fields(self, i, q=None):
        q = self.sim.get_fields() if q is None else q
        return q[self.offsets[i]:self.offsets[i + 1]]

    def standalone_pml(self, i) -> dict:
        r = self.recipe[i]
        return dict(self.cfg["pml"], sigma_max=[r["sigma_max"]] * 3, order=r["order"])
