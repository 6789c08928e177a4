"""Seeded batches of independent simulations (inputs only: no DG or PML arithmetic).

A batch recipe draws, per simulation, the mesh resolution n (an n^3 x 6 Kuhn
box), the absorbing-layer sigma_max and profile order, and a mesh seed; the
meshes are then concatenated with disjoint vertex sets, so that no face is
shared between simulations.
"""
from __future__ import annotations

import numpy as np

from .mesh import kuhn_box


def batch_recipe(spec: dict) -> list:
    """Per-simulation parameters from a batch spec: nsim, n_range [lo, hi], sigma_range [lo, hi],
    orders (list), seed."""
    rng = np.random.default_rng(spec["seed"])
    n_lo, n_hi = spec["n_range"]
    s_lo, s_hi = spec["sigma_range"]
    out = []
    for _ in range(spec["nsim"]):
        out.append({"n": int(rng.integers(n_lo, n_hi + 1)),
                    "sigma_max": float(rng.uniform(s_lo, s_hi)),
                    "order": float(rng.choice(spec["orders"])),
                    "mesh_seed": int(rng.integers(0, 2 ** 31 - 1))})
    return out


def batch_meshes(cfg: dict, recipe: list) -> list:
    """One (vxyz, etov) per simulation on the recipe's box."""
    m = cfg["mesh"]
    return [kuhn_box(r["n"], m["lo"], m["hi"], m.get("perturb", 0.0), r["mesh_seed"]) for r in recipe]


def concat_meshes(meshes: list):
    """Disjoint union: (vxyz, etov, group [K] int32, offsets [nsim + 1] element offsets)."""
    vx, ev, group, offsets = [], [], [], [0]
    nv = 0
    for g, (v, e) in enumerate(meshes):
        vx.append(v)
        ev.append(np.asarray(e, dtype=np.int64) + nv)
        group.append(np.full(len(e), g, dtype=np.int32))
        nv += len(v)
        offsets.append(offsets[-1] + len(e))
    return (np.concatenate(vx), np.concatenate(ev).astype(np.int32), np.concatenate(group),
            np.asarray(offsets, dtype=np.int64))
