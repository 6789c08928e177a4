"""Generator of fully symmetric positive interior cubature rules on a tetrahedron.

The weight-adjusted mass matrices of the method are formed by a cubature rule
of degree 2N (the paper's practice, Sec. III) or 2N+2 on the reference
tetrahedron.  The paper takes its rules from published tables that are not
available here, so this module builds its own rules, which are then stored as
plain text next to this file and read by both the library caller and the test
oracle like any other input.

Construction (moment fitting): the nodes are unions of orbits of the symmetry
group of the tetrahedron, written in barycentric coordinates
(l0, l1, l2, l3):

    S4    (1/4, 1/4, 1/4, 1/4)                 1 point,  0 shape parameters
    S31   (a, a, a, 1-3a)                      4 points, 1
    S22   (a, a, 1/2-a, 1/2-a)                 6 points, 1
    S211  (a, a, b, 1-2a-b)                   12 points, 2
    S1111 (a, b, c, 1-a-b-c)                  24 points, 3

with one weight per orbit.  The shape parameters and weights are fitted by
Levenberg-Marquardt so that every barycentric monomial l1^i l2^j l3^k with
i+j+k <= D is integrated exactly over the reference tetrahedron
(exact value 8 i! j! k! / (i+j+k+3)!; the reference tetrahedron with vertices
(-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1) is 8 times the unit simplex).
Random restarts are kept only if all weights are positive, all points lie
strictly inside, and the moment residual is at rounding level.

Run ``python -m paper_2006_02551_amd.inputs.cubature_gen`` to regenerate the
stored files ``cubature/tet_deg{D}.txt`` (columns r s t w, reference
coordinates, weights summing to 4/3).
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
from scipy.optimize import least_squares

HERE = os.path.dirname(os.path.abspath(__file__))
DATA_DIR = os.path.join(HERE, "cubature")

NPARAM = {"S4": 0, "S31": 1, "S22": 1, "S211": 2, "S1111": 3}
NPTS = {"S4": 1, "S31": 4, "S22": 6, "S211": 12, "S1111": 24}


def _orbit(kind: str, p) -> np.ndarray:
    if kind == "S4":
        base = (0.25, 0.25, 0.25, 0.25)
    elif kind == "S31":
        a = p[0]
        base = (a, a, a, 1.0 - 3.0 * a)
    elif kind == "S22":
        a = p[0]
        base = (a, a, 0.5 - a, 0.5 - a)
    elif kind == "S211":
        a, b = p
        base = (a, a, b, 1.0 - 2.0 * a - b)
    elif kind == "S1111":
        a, b, c = p
        base = (a, b, c, 1.0 - a - b - c)
    else:
        raise ValueError(kind)
    # Distinct permutations, found on integer labels so that equal parameter
    # values do not change the point count.
    labels = {"S4": (0, 0, 0, 0), "S31": (0, 0, 0, 1), "S22": (0, 0, 1, 1),
              "S211": (0, 0, 1, 2), "S1111": (0, 1, 2, 3)}[kind]
    seen = set()
    pts = []
    for perm in itertools.permutations(range(4)):
        lab = tuple(labels[i] for i in perm)
        if lab in seen:
            continue
        seen.add(lab)
        pts.append([base[i] for i in perm])
    return np.asarray(pts)


def _monomials(D: int):
    return [(i, j, k) for i in range(D + 1) for j in range(D + 1 - i) for k in range(D + 1 - i - j)]


def exact_moment(i: int, j: int, k: int) -> float:
    """Integral of l1^i l2^j l3^k over the reference tetrahedron (volume 4/3)."""
    return 8.0 * math.factorial(i) * math.factorial(j) * math.factorial(k) / math.factorial(i + j + k + 3)


def _unpack(x, structure):
    pts, wts = [], []
    pos = 0
    for kind in structure:
        npar = NPARAM[kind]
        p = x[pos:pos + npar]
        w = x[pos + npar]
        pos += npar + 1
        o = _orbit(kind, p)
        pts.append(o)
        wts.append(np.full(len(o), w))
    return np.vstack(pts), np.concatenate(wts)


def _residual(x, structure, mons, exact):
    lam, w = _unpack(x, structure)
    l1, l2, l3 = lam[:, 1], lam[:, 2], lam[:, 3]
    vals = np.stack([l1 ** i * l2 ** j * l3 ** k for (i, j, k) in mons], axis=0)
    return (vals @ w - exact) / exact


def _random_start(structure, rng, npts):
    x = []
    for kind in structure:
        if kind == "S31":
            x.append(rng.uniform(0.0, 1.0 / 3.0))
        elif kind == "S22":
            x.append(rng.uniform(0.0, 0.5))
        elif kind == "S211":
            a = rng.uniform(0.0, 0.5)
            x += [a, rng.uniform(0.0, 1.0 - 2.0 * a)]
        elif kind == "S1111":
            v = rng.dirichlet(np.ones(4))
            x += list(v[:3])
        x.append(rng.uniform(0.5, 1.5) * (4.0 / 3.0) / npts)
    return np.asarray(x)


def fit(D: int, structure, tries: int = 4000, seed: int = 0, stop_after: int = 8):
    """Search for a positive interior rule of degree D with the given orbit structure."""
    mons = _monomials(D)
    exact = np.array([exact_moment(*m) for m in mons])
    npts = sum(NPTS[k] for k in structure)
    rng = np.random.default_rng(seed)
    best = None
    found = 0
    for _ in range(tries):
        x0 = _random_start(structure, rng, npts)
        try:
            sol = least_squares(_residual, x0, args=(structure, mons, exact), method="lm",
                                xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=4000)
        except Exception:
            continue
        res = np.max(np.abs(sol.fun))
        if res > 1e-13:
            continue
        lam, w = _unpack(sol.x, structure)
        if np.min(w) <= 0 or np.min(lam) <= 1e-6:
            continue
        score = np.min(lam)  # prefer points away from the boundary
        found += 1
        if best is None or score > best[0]:
            best = (score, lam, w, res)
        if found >= stop_after:
            break
    if best is None:
        return None
    _, lam, w, res = best
    rst = -1.0 + 2.0 * lam[:, 1:4]
    return rst, w, res


# Orbit structures tried per degree, fewest points first.
STRUCTURES = {
    2: [("S31",)],
    4: [("S31", "S31", "S22")],
    6: [("S31", "S31", "S31", "S211")],
    8: [("S4", "S31", "S31", "S31", "S22", "S211", "S211"),
        ("S31", "S31", "S31", "S31", "S31", "S211", "S211"),
        ("S4", "S31", "S31", "S22", "S211", "S211", "S211")],
}


def write_rule(D: int, rst: np.ndarray, w: np.ndarray, path: str) -> None:
    with open(path, "w") as fh:
        fh.write(f"# fully symmetric positive interior tetrahedron rule, degree {D}, {len(w)} points\n")
        fh.write("# reference tet (-1,-1,-1) (1,-1,-1) (-1,1,-1) (-1,-1,1); columns r s t w; sum w = 4/3\n")
        for p, wq in zip(rst, w):
            fh.write(f"{float(p[0]):.17e} {float(p[1]):.17e} {float(p[2]):.17e} {float(wq):.17e}\n")


def main():
    os.makedirs(DATA_DIR, exist_ok=True)
    for D, cands in STRUCTURES.items():
        for st in cands:
            out = fit(D, st, tries=400 if D < 8 else 3000)
            if out is None:
                print(f"degree {D}: structure {st} found no positive interior rule")
                continue
            rst, w, res = out
            path = os.path.join(DATA_DIR, f"tet_deg{D}.txt")
            write_rule(D, rst, w, path)
            print(f"degree {D}: {len(w)} points, max rel residual {res:.2e}, min weight {w.min():.3e} -> {path}")
            break


if __name__ == "__main__":
    main()
