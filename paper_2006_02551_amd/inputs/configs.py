"""Workload recipes: synthetic stand-ins for the paper's experiments.

The paper measures on a plane-wave box and a PEC-sphere mesh (Sec. III) that
are not available; these seeded cube meshes with a six-sided absorbing layer
stand in for them.  Their PML fraction (70-90% of elements) is close to the
72% of the paper's Table I workload.

Each recipe is a plain dict:

  N           polynomial order
  cub_degree  cubature degree (2N in the paper's Sec. III, 2N+2 for c1)
  mesh        Kuhn box: n (cubes per side), lo, hi, perturb (fraction of h), seed
  pml         interface box lo/hi, thickness L, sigma_max (per axis), order p,
              kappa_max
  alpha       flux upwinding (1 upwind, 0 central)
  init        Gaussian initial field: component (0..5 = Ex..Hz), center, width
  source      Gaussian-modulated dipole current (or None):
              amplitude * sin(2 pi f0 (t-t0)) exp(-((t-t0)/tau)^2)
              * exp(-|x-center|^2/width^2) * direction
  probes      probe points [n, 3] (or None)
  steps       number of LSERK4 steps
  shell       (differentiation form) box shell of the loss: outer_lo/hi, inner_lo/hi
  batch       (batching form) nsim, n_range, sigma_range, orders, seed of the per-simulation draws;
              the recipe's mesh box, PML box and thickness are shared
  column      (reflection study) Kuhn grid n[3], lo[3], hi[3], perturb, seed, periodic[3]
  plane_pulse (reflection study) right-going Gaussian plane pulse E_x = H_y = exp(-((z-z0)/width)^2)
  cfl         dt = cfl / ((N+1)^2 * max_{k,f} Fscale_{k,f})
"""
from __future__ import annotations

import copy
import os

import numpy as np

from .mesh import kuhn_box, kuhn_grid

HERE = os.path.dirname(os.path.abspath(__file__))
RULE_DIR = os.path.join(HERE, "cubature")

_CUBE8 = [[sx * 0.5, sy * 0.5, sz * 0.5] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]

_DIPOLE = {"amplitude": 1.0, "f0": 1.0, "t0": 0.75, "tau": 0.25, "center": [0.0, 0.0, 0.0],
           "width": 0.15, "direction": [0.0, 0.0, 1.0]}

CFL = 0.75

CONFIGS = {
    # 384 tets, N=2, quadratic profile sigma_max=20, Gaussian Ez pulse, 100 steps.
    "c1": {"name": "c1", "N": 2, "cub_degree": 6,
           "mesh": {"n": 4, "lo": -1.0, "hi": 1.0, "perturb": 0.0, "seed": 0},
           "pml": {"lo": [-0.5] * 3, "hi": [0.5] * 3, "L": [0.5] * 3, "sigma_max": [20.0] * 3,
                   "order": 2.0, "kappa_max": 1.0},
           "alpha": 1.0,
           "init": {"component": 2, "center": [0.0, 0.0, 0.0], "width": 0.2},
           "source": None, "probes": None, "steps": 100, "cfl": CFL},
    # 48,000 perturbed tets, N=3, cubic profile sigma_max=30, dipole, 8 probes, 1000 steps.
    "c2": {"name": "c2", "N": 3, "cub_degree": 6,
           "mesh": {"n": 20, "lo": -1.5, "hi": 1.5, "perturb": 0.1, "seed": 0},
           "pml": {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [30.0] * 3,
                   "order": 3.0, "kappa_max": 1.0},
           "alpha": 1.0, "init": None, "source": _DIPOLE, "probes": _CUBE8, "steps": 1000, "cfl": CFL},
    # 384,000 perturbed tets, N=4, quadratic profile sigma_max=40, dipole, 2000 steps.
    "c3": {"name": "c3", "N": 4, "cub_degree": 8,
           "mesh": {"n": 40, "lo": -1.5, "hi": 1.5, "perturb": 0.1, "seed": 0},
           "pml": {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [40.0] * 3,
                   "order": 2.0, "kappa_max": 1.0},
           "alpha": 1.0, "init": None, "source": _DIPOLE, "probes": _CUBE8, "steps": 2000, "cfl": CFL},
    # Batching form: 32 independent simulations in one launch, meshes 8^3 x 6 .. 24^3 x 6, each with its own
    # sigma_max in [10, 50] and profile order in {2, 3, 4}, N=3, FP32, 500 steps, a Gaussian Ez pulse each.
    "c4": {"name": "c4", "N": 3, "cub_degree": 6,
           "mesh": {"n": 0, "lo": -1.5, "hi": 1.5, "perturb": 0.1, "seed": 0},
           "pml": {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [30.0] * 3,
                   "order": 3.0, "kappa_max": 1.0},
           "alpha": 1.0, "init": {"component": 2, "center": [0.0, 0.0, 0.0], "width": 0.25},
           "source": None, "probes": None, "steps": 500, "cfl": CFL,
           "batch": {"nsim": 32, "n_range": [8, 24], "sigma_range": [10.0, 50.0], "orders": [2, 3, 4], "seed": 0}},
    # Table I stand-in: 23^3 x 6 = 73,002 perturbed tets (52,752 in the PML, 72.3%; Table I: 72,762 and
    # 52,657), the c2 box and cubic profile; the order N is scanned 1..4 with cubature of degree 2N.
    "t1": {"name": "t1", "N": 3, "cub_degree": 6,
           "mesh": {"n": 23, "lo": -1.5, "hi": 1.5, "perturb": 0.1, "seed": 0},
           "pml": {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [30.0] * 3,
                   "order": 3.0, "kappa_max": 1.0},
           "alpha": 1.0, "init": {"component": 2, "center": [0.0, 0.0, 0.0], "width": 0.25},
           "source": None, "probes": None, "steps": 50, "cfl": CFL},
    # Plane-wave reflection study (normal incidence, Sec. III, Fig. 2): a column periodic in x and y,
    # 3 x 3 x 60 cubes x 6 = 3,240 tets of edge 0.1 over [0, 0.3]^2 x [0, 6] with interior vertices
    # perturbed by up to 20% of h (element faces do not follow the layer: a "paved" mesh), PML slabs
    # z < 1 and z > 5 of thickness 1 ended by PEC walls, quadratic profile; a right-going Gaussian plane
    # pulse E_x = H_y centred at z = 2 is the initial state, E_x is recorded at z = 3 until t = 8 (the
    # incident pulse passes at t = 1, the interface reflection returns at t = 5, the wall's at t = 7).
    "x1": {"name": "x1", "N": 3, "cub_degree": 6,
           "column": {"n": [3, 3, 60], "lo": [0.0, 0.0, 0.0], "hi": [0.3, 0.3, 6.0], "perturb": 0.2, "seed": 0,
                      "periodic": [True, True, False]},
           "pml": {"lo": [-1e9, -1e9, 1.0], "hi": [1e9, 1e9, 5.0], "L": [1.0, 1.0, 1.0],
                   "sigma_max": [0.0, 0.0, 20.0], "order": 2.0, "kappa_max": 1.0},
           "alpha": 1.0, "plane_pulse": {"z0": 2.0, "width": 0.2}, "probe": [0.15, 0.15, 3.0],
           "t_end": 8.0, "t_split": 2.5, "source": None, "probes": None, "cfl": CFL,
           "scan": {"sigma_max": [1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0, 256.0, 512.0], "N": [2, 3, 4]}},
    # Differentiation form: the 48,000-tet N=3 mesh and cubic profile of c2, a Gaussian Ez pulse at the
    # origin that reaches the layer within the 500 steps, loss = time-integrated energy in the shell
    # 0.1 inside the PML interface.
    "c5": {"name": "c5", "N": 3, "cub_degree": 6,
           "mesh": {"n": 20, "lo": -1.5, "hi": 1.5, "perturb": 0.1, "seed": 0},
           "pml": {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [30.0] * 3,
                   "order": 3.0, "kappa_max": 1.0},
           "alpha": 1.0, "init": {"component": 2, "center": [0.0, 0.0, 0.0], "width": 0.25},
           "source": None, "probes": None, "steps": 500, "cfl": CFL,
           "shell": {"outer_lo": [-1.0] * 3, "outer_hi": [1.0] * 3, "inner_lo": [-0.9] * 3, "inner_hi": [0.9] * 3}},
}


def config(name: str, **overrides) -> dict:
    """Deep copy of a recipe with top-level or nested ('mesh.n') overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    for key, val in overrides.items():
        parts = key.split(".")
        d = cfg
        for p in parts[:-1]:
            d = d[p]
        d[parts[-1]] = val
    return cfg


def mesh_for(cfg: dict):
    m = cfg["mesh"]
    return kuhn_box(m["n"], m["lo"], m["hi"], m.get("perturb", 0.0), m.get("seed", 0))


def column_for(cfg: dict):
    """(vxyz, etov, vertex_id) of a recipe's periodic column."""
    c = cfg["column"]
    return kuhn_grid(c["n"], c["lo"], c["hi"], c.get("perturb", 0.0), c.get("seed", 0), tuple(c["periodic"]))


def plane_pulse_fields(cfg: dict, xnodes: np.ndarray) -> np.ndarray:
    """Right-going plane pulse E_x = H_y = exp(-((z - z0)/width)^2), state [K, 12, N_p]."""
    p = cfg["plane_pulse"]
    g = np.exp(-(((xnodes[..., 2] - p["z0"]) / p["width"]) ** 2))
    q = np.zeros((xnodes.shape[0], 12, xnodes.shape[1]))
    q[:, 0] = g
    q[:, 4] = g
    return q


def load_rule(degree: int):
    """Stored cubature rule of the given degree: (rst [Nq, 3], w [Nq])."""
    data = np.loadtxt(os.path.join(RULE_DIR, f"tet_deg{degree}.txt"), comments="#")
    data = np.atleast_2d(data)
    return np.ascontiguousarray(data[:, :3]), np.ascontiguousarray(data[:, 3])


def product_rule(n: int):
    """Conical product rule with n^3 points on the reference tetrahedron, exact to polynomial degree 2n - 1.

    Collapsed coordinates (a, b, c) in [-1, 1]^3 map to the tetrahedron with vertices (-1,-1,-1), (1,-1,-1),
    (-1,1,-1), (-1,-1,1) by r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c, whose Jacobian is
    (1-b)(1-c)^2/8; Gauss rules for the weights 1, (1-b) and (1-c)^2 absorb it.  Used for integrals
    whose integrand is not a low-degree polynomial (profile-weighted mass matrices).
    Returns (rst [n^3, 3], w [n^3]); the weights sum to 4/3.
    """
    from scipy.special import roots_jacobi

    a, wa = roots_jacobi(n, 0.0, 0.0)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, Bc, Cc = np.meshgrid(a, b, c, indexing="ij")
    W = np.einsum("i,j,k->ijk", wa, wb, wc) / 8.0
    r = (1.0 + A) * (1.0 - Bc) * (1.0 - Cc) / 4.0 - 1.0
    s = (1.0 + Bc) * (1.0 - Cc) / 2.0 - 1.0
    rst = np.stack([r.ravel(), s.ravel(), Cc.ravel()], axis=1)
    return np.ascontiguousarray(rst), np.ascontiguousarray(W.ravel())


def gaussian_fields(cfg: dict, xnodes: np.ndarray) -> np.ndarray:
    """Initial state [K, 12, N_p] from node coordinates xnodes [K, N_p, 3]."""
    K, Np, _ = xnodes.shape
    q = np.zeros((K, 12, Np))
    init = cfg.get("init")
    if init:
        r2 = np.sum((xnodes - np.asarray(init["center"])) ** 2, axis=-1)
        q[:, init["component"], :] = np.exp(-r2 / init["width"] ** 2)
    return q
